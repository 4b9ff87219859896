"""Pins for the layer schedules (CPU only).

1. The nine special-convolution masks (closed form) have the structure
   Algorithms 2/3 give them, and a hand-worked W = 3 case.
2. Every schedule, run as a plain float slot simulation, equals the paper's
   FP64 layer equation (direct loops), and uses the documented number of key
   switches and levels.
3. The same schedules under the oracle's CKKS arithmetic decrypt to the FP64
   result within the stated tolerance (1e-3 per layer, 1e-2 for the LeNet-5
   shaped stack) at the real ring sizes.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import ckks
from oracle import layers as LY
from tests import helpers as H

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# Algorithm 3 of the special convolution builds tap k's mask with Algorithm 2
# from three numbers: sp leading zeros, ep trailing zeros, and in between runs
# of w ones each followed by one zero (m = W^2 entries per channel).  These
# are the paper's (sp, ep, w) per tap k = 3 (dy + 1) + (dx + 1), as functions
# of W (m = W^2 stands for "one run over the whole block").
def _alg3_params(W):
    m = W * W
    return [(W + 1, 0, W - 1), (W, 0, m), (W, 0, W - 1), (1, 0, W - 1), (0, 0, m),
            (0, 1, W - 1), (1, W - 1, W - 1), (0, W, m), (0, W + 1, W - 1)]


@pytest.mark.parametrize("W", [3, 4, 5, 8, 32])
@pytest.mark.parametrize("C", [1, 3])
def test_special_masks_have_the_alg3_structure(W, C):
    """The closed-form masks equal the structure Algorithm 2 describes for
    Algorithm 3's parameters: zero on the first sp and the last ep entries,
    and at offset t >= sp one unless (t - sp) is the last position of a run
    of w ones; repeated once per input channel."""
    m = W * W
    got = LY.special_masks(W, C)
    for k, (sp, ep, w) in enumerate(_alg3_params(W)):
        want = np.zeros(m)
        for t in range(sp, m - ep):
            want[t] = 0.0 if (t - sp) % (w + 1) == w else 1.0
        assert np.array_equal(got[k], np.tile(want, C)), (W, k)


def test_special_masks_worked_example_w3():
    """W = 3 worked by hand from the zero-padded 3x3 convolution: tap (dy, dx)
    contributes to output (y, x) only if (y + dy, x + dx) is inside the image."""
    want = [
        [0, 0, 0, 0, 1, 1, 0, 1, 1], [0, 0, 0, 1, 1, 1, 1, 1, 1], [0, 0, 0, 1, 1, 0, 1, 1, 0],
        [0, 1, 1, 0, 1, 1, 0, 1, 1], [1, 1, 1, 1, 1, 1, 1, 1, 1], [1, 1, 0, 1, 1, 0, 1, 1, 0],
        [0, 1, 1, 0, 1, 1, 0, 0, 0], [1, 1, 1, 1, 1, 1, 0, 0, 0], [1, 1, 0, 1, 1, 0, 0, 0, 0],
    ]
    got = LY.special_masks(3, 1)
    for k in range(9):
        assert got[k].tolist() == want[k], k
    # ones per tap: (W - |dy|) (W - |dx|)
    for W in (4, 7):
        for k, mk in enumerate(LY.special_masks(W, 1)):
            dy, dx = k // 3 - 1, k % 3 - 1
            assert mk.sum() == (W - abs(dy)) * (W - abs(dx))


def test_paper_output_size_formulas():
    """Output-size equations (Secure Advanced Convolution) on the layer shapes
    of the paper's architecture tables (fixture cites the tables)."""
    fx = json.load(open(os.path.join(GOLDEN, "paper_layer_shapes.json")))
    for row in fx["layers"]:
        H_in, k, S, P = row["in_hw"], row["kernel"], row["stride"], row["padding"]
        assert (H_in + 2 * P - k) // S + 1 == row["out_hw"], row
    fc = fx["lenet5_fc_input"]
    assert fc["channels"] * fc["hw"] ** 2 == fc["fc_in"]


def sim(slots):
    return LY.SimEval(slots)


def test_sim_config0_special_conv():
    X = synth.image(1, 1, 8, 8)
    K = synth.conv_weights(1, 1, 1, 3, 0.1)
    fm = LY.FMap(1, 8, 8)
    slots = 2048
    kern, masks = LY.conv_plaintexts(fm, K, 1, 1, slots)
    ev = sim(slots)
    y, fo = LY.conv2d(ev, LY.SimCt(LY.pack(X, fm, slots), 3), fm, 1, 3, 1, 1, kern, masks, slots)
    assert ev.ks == 8 and y.level == 2
    assert np.max(np.abs(LY.unpack(y.v, fo) - LY.conv2d_ref(X, K, 1, 1))) < 1e-12


@pytest.mark.parametrize("stride,F", [(1, 16), (2, 32)])
def test_sim_config2_special_conv(stride, F):
    slots = 32768
    X = synth.image(2, 16, 32, 32)
    K = synth.conv_weights(2, F, 16, 3, (2.0 / 144) ** 0.5)
    fm = LY.FMap(16, 32, 32, reps=2)
    kern, masks = LY.conv_plaintexts(fm, K, stride, 1, slots)
    ev = sim(slots)
    y, fo = LY.conv2d(ev, LY.SimCt(LY.pack(X, fm, slots), 24), fm, F, 3, stride, 1, kern, masks, slots)
    ref = LY.conv2d_ref(X, K, stride, 1)
    assert np.max(np.abs(LY.unpack(y.v, fo) - ref)) < 1e-9
    if stride == 1:
        assert ev.ks == 248 and 24 - y.level == 2 and fo.reps == 2
        # replication preserved: the second copy equals the first
        assert np.array_equal(y.v[:16384], y.v[16384:])
    else:
        assert ev.ks == 549 and 24 - y.level == 5 and fo == LY.FMap(32, 16, 16)
    assert len(LY.conv_rotations(fm, F, 3, stride, 1, slots)) == (5 if stride == 1 else 7)


def test_sim_config1_stack():
    """conv 5x5 1->6 -> degree-4 ReLU polynomial -> 2x2 average pool, 7 levels."""
    slots = 8192
    X = synth.image(3, 1, 28, 28)
    K = synth.conv_weights(3, 6, 1, 5, 0.1)
    fm = LY.FMap(1, 28, 28)
    kern, masks = LY.conv_plaintexts(fm, K, 1, 0, slots)
    ev = sim(slots)
    y, f1 = LY.conv2d(ev, LY.SimCt(LY.pack(X, fm, slots), 8), fm, 6, 5, 1, 0, kern, masks, slots)
    assert f1 == LY.FMap(6, 24, 24, 28, 784) and ev.ks == 29 and y.level == 7
    ref = LY.conv2d_ref(X, K, 1, 0)
    assert np.max(np.abs(LY.unpack(y.v, f1) - ref)) < 1e-12
    p = LY.relu_poly4(ev, y, 2.0 ** 45)
    assert p.level == 4 and ev.ks == 29
    ref = LY.relu4_ref(ref)
    assert np.max(np.abs(LY.unpack(p.v, f1) - ref)) < 1e-12
    pm = LY.avgpool_plaintexts(f1, 2, 2, slots)
    z, f2 = LY.avgpool(ev, p, f1, 2, 2, pm)
    assert f2 == LY.FMap(6, 12, 12) and z.level == 1 and ev.ks == 59
    assert np.max(np.abs(LY.unpack(z.v, f2) - LY.avgpool_ref(ref, 2, 2))) < 1e-12


@pytest.mark.parametrize("C,HW,ks", [(32, 16, 39), (64, 8, 69)])
def test_sim_gap(C, HW, ks):
    slots = 32768
    X = synth.image(4, C, HW, HW)
    fm = LY.FMap(C, HW, HW)
    ev = sim(slots)
    y, fo = LY.gap(ev, LY.SimCt(LY.pack(X, fm, slots), 10), fm, LY.gap_plaintexts(fm, slots))
    assert ev.ks == ks and y.level == 9
    assert np.max(np.abs(y.v[:C] - LY.gap_ref(X))) < 1e-12 and np.max(np.abs(y.v[C:])) < 1e-12


@pytest.mark.parametrize("C,HW", [(4, 8), (16, 4), (2, 16)])
def test_sim_pool_whole_channel(C, HW):
    """The pooling special case: a k = H = W window is the global schedule
    (log2(H W) sum rotations plus a one-key gather, not k^2 - 1 window
    rotations and a compaction) and still equals the window average."""
    slots = 8192
    X = synth.image(7, C, HW, HW)
    fm = LY.FMap(C, HW, HW)
    assert LY.pool_whole_channel(fm, HW) and not LY.pool_whole_channel(fm, HW - 1)
    assert not LY.pool_whole_channel(LY.FMap(C, HW, HW, 2 * HW, 2 * HW * HW), HW)
    ev = sim(slots)
    pm = LY.avgpool_plaintexts(fm, HW, HW, slots)
    assert len(pm) == C
    y, fo = LY.avgpool(ev, LY.SimCt(LY.pack(X, fm, slots), 10), fm, HW, HW, pm)
    steps = int(np.log2(HW * HW))
    assert fo == LY.FMap(C, 1, 1, 1, 1, 1) and y.level == 9 and ev.ks == steps + C - 1
    ref = LY.avgpool_ref(X, HW, HW)
    assert np.max(np.abs(LY.unpack(y.v, fo) - ref)) < 1e-12 and np.max(np.abs(y.v[C:])) < 1e-12
    keys = LY.avgpool_rotations(fm, HW, HW)
    assert keys == sorted({1 << t for t in range(steps)} | {HW * HW - 1})


def test_sim_fc():
    slots = 32768
    x = np.zeros(64)
    x[:32] = synth.uniform_slots(5, 32)
    Wm = synth.fc_weights(5, 10, 64, (2.0 / 64) ** 0.5)
    v = np.zeros(slots)
    v[:64] = x
    rows, masks = LY.fc_plaintexts(Wm, slots)
    ev = sim(slots)
    y = LY.fc(ev, LY.SimCt(v, 10), 64, 10, rows, masks)
    assert ev.ks == 69 and y.level == 8
    assert np.max(np.abs(y.v[:10] - LY.fc_ref(x, Wm))) < 1e-12 and np.max(np.abs(y.v[10:])) < 1e-12


def test_sim_generic_conv_multichannel_stride():
    """Generic convolution with C > 1 and stride 2 (block-0 mask + placement + compaction)."""
    slots = 4096
    X = synth.image(6, 3, 12, 12)
    K = synth.conv_weights(6, 4, 3, 3, 0.2)
    fm = LY.FMap(3, 12, 12)
    kern, masks = LY.conv_plaintexts(fm, K, 2, 0, slots)
    ev = sim(slots)
    y, fo = LY.conv2d(ev, LY.SimCt(LY.pack(X, fm, slots), 12), fm, 4, 3, 2, 0, kern, masks, slots)
    assert fo == LY.FMap(4, 5, 5)
    assert np.max(np.abs(LY.unpack(y.v, fo) - LY.conv2d_ref(X, K, 2, 0))) < 1e-12


@pytest.mark.parametrize("C,F,HW,k,S,P", [
    (2, 3, 12, 5, 1, 2),   # 5x5 "same" padding
    (3, 2, 16, 7, 2, 3),   # the ResNet-34 stem shape 7x7 / s2 / p3
    (2, 2, 12, 3, 1, 1),   # 3x3 / p1 on a non-replicated multi-channel map
    (3, 4, 12, 3, 2, 1),
    (1, 1, 10, 5, 2, 1),   # padding below (k-1)/2
    (2, 2, 9, 1, 1, 0),    # 1x1
])
def test_sim_generic_conv_with_padding(C, F, HW, k, S, P):
    """Zero padding by masked taps equals the FP64 convolution with padding P."""
    slots = 4096
    X = synth.image(7, C, HW, HW)
    K = synth.conv_weights(7, F, C, k, 0.2)
    fm = LY.FMap(C, HW, HW)
    assert LY.conv_kind(k, P, fm, F) == "generic"
    kern, masks = LY.conv_plaintexts(fm, K, S, P, slots)
    ev = sim(slots)
    y, fo = LY.conv2d(ev, LY.SimCt(LY.pack(X, fm, slots), 12), fm, F, k, S, P, kern, masks, slots)
    Ho = (HW + 2 * P - k) // S + 1
    assert (fo.C, fo.H, fo.W) == (F, Ho, Ho) and fo == LY.conv_out_map(fm, F, k, S, P, slots)
    assert np.max(np.abs(LY.unpack(y.v, fo) - LY.conv2d_ref(X, K, S, P))) < 1e-12
    # rotations: k^2 - 1 taps, C - 1 per out-channel for the channel sum, F - 1 placements, compaction
    taps = k * k - 1
    assert ev.ks >= taps + F * (C - 1) + (F - 1 if F > 1 else 0)
    keys = LY.conv_rotations(fm, F, k, S, P, slots)
    assert {(i - P) * HW + (j - P) for i in range(k) for j in range(k)} - {0} <= set(keys)


STRIDE_MAPS = [  # (C, H1, W1, rs, cs, S)
    (1, 32, 32, 32, 1024, 2),   # ResNet downsampling: Wo = 16 (power of two)
    (3, 12, 12, 12, 144, 2),    # Wo = 6
    (2, 11, 13, 16, 200, 3),    # S = 3, Wo = 5, padded row stride
    (4, 9, 9, 9, 81, 2),        # Wo = 5
    (2, 3, 2, 4, 16, 2),        # Wo = 1: no column step
    (1, 5, 17, 17, 85, 4),      # S = 4, Wo = 5
]


@pytest.mark.parametrize("C,H1,W1,rs,cs,S", STRIDE_MAPS)
@pytest.mark.parametrize("bsgs", [False, True], ids=["horner", "bsgs"])
def test_log_step_striding_equals_extraction(C, H1, W1, rs, cs, S, bsgs):
    """Striding approach 2 (ceil(log2 Wo) column steps with keys (S-1) 2^t)
    moves every stride-aligned output exactly where approach 1 does, from a
    ciphertext full of values (every slot nonzero), with log2(Wo) + 1 keys
    for one channel and ceil(log2 Wo) column key switches instead of Wo - 1."""
    slots = 4096
    rng = np.random.default_rng(11)
    v = rng.uniform(-1, 1, slots)
    fm = LY.FMap(C, H1, W1, rs, cs)
    Ho, Wo = (H1 - 1) // S + 1, (W1 - 1) // S + 1
    out = []
    for log in (False, True):
        ev = sim(slots)
        masks = LY.compaction_masks(fm, S, Ho, Wo, 0.25, slots, bsgs, log)
        y, fo = LY.compaction(ev, LY.SimCt(v, 9), fm, S, Ho, Wo, masks, bsgs, log)
        out.append((y, fo, ev.ks))
    (y1, f1, ks1), (y2, f2, ks2) = out
    assert f1 == f2 == LY.FMap(C, Ho, Wo, Wo, Ho * Wo)
    assert np.array_equal(y1.v, y2.v)
    want = np.zeros(slots)
    for c in range(C):
        for i in range(Ho):
            for j in range(Wo):
                want[c * Ho * Wo + i * Wo + j] = 0.25 * v[c * cs + S * i * rs + S * j]
    assert np.array_equal(y2.v, want)
    T = LY.log_steps(Wo)
    assert T == int(np.ceil(np.log2(Wo))) if Wo > 1 else T == 0
    rest = sum(LY.masked_chain_switches(n, bsgs) for st, n, _ in LY.compaction_plan(fm, S, Ho, Wo) if st != "col")
    assert ks2 == (T if Wo > 1 else 0) + rest and ks1 == LY.masked_chain_switches(Wo, bsgs) + rest
    assert y2.level == 9 - (max(T, 1) + len(LY.compaction_plan(fm, S, Ho, Wo)) - 1)
    keys = LY.compaction_keys(fm, S, Ho, Wo, False, True)
    if C == 1 and Ho > 1 and Wo > 1:
        assert len(keys) == T + 1 and {(S - 1) << t for t in range(T)} <= keys


@pytest.mark.parametrize("C,g", [(6, 2), (7, 3), (4, 4), (5, 1), (3, 0)])
@pytest.mark.parametrize("log", [False, True], ids=["extract", "logstride"])
def test_grouped_striding_equals_joint(C, g, log):
    """The multi-channel pipeline (groups of g channels, each compacted
    jointly, merged with the key g E) places every output exactly where the
    all-channel compaction does, from a ciphertext with every slot nonzero;
    (G - 1) merge key switches on top of G group compactions."""
    slots = 4096
    v = np.random.default_rng(12).uniform(-1, 1, slots)
    fm = LY.FMap(C, 9, 9, 12, 120)
    S, Ho, Wo = 2, 5, 5
    ev1, ev2 = sim(slots), sim(slots)
    joint, _ = LY.compaction(ev1, LY.SimCt(v, 9), fm, S, Ho, Wo,
                             LY.compaction_masks(fm, S, Ho, Wo, 1.0, slots, False, log), False, log)
    grp, fo = LY.strided(ev2, LY.SimCt(v, 9), fm, S, Ho, Wo,
                         LY.strided_masks(fm, S, Ho, Wo, 1.0, slots, False, log, g), False, log, g)
    assert fo == LY.FMap(C, Ho, Wo) and np.array_equal(joint.v, grp.v) and grp.level == joint.level
    groups = LY.stride_groups(C, g)
    per = lambda n: sum(LY.masked_chain_switches(k, False)
                        for _, k, _ in LY.compaction_plan(LY.FMap(n, 9, 9, 12, 120), S, Ho, Wo, log, C > 1))
    assert ev2.ks == sum(per(n) for _, n in groups) + len(groups) - 1
    keys = LY.strided_keys(fm, S, Ho, Wo, False, log, g)
    assert (g * (120 - Ho * Wo) in keys) == (len(groups) > 1)


def test_conv_b_with_the_paper_grouping():
    """ResNet conv B (16 -> 32, 3x3, stride 2, pad 1) with groups of g = 16
    (the layer's input channels): 579 key switches against the joint
    compaction's 549, the same FP64 result."""
    slots = 32768
    X = synth.image(2, 16, 32, 32)
    K = synth.conv_weights(2, 32, 16, 3, 0.1)
    fm = LY.FMap(16, 32, 32, reps=2)
    out = []
    for g in (0, 16):
        kern, masks = LY.conv_plaintexts(fm, K, 2, 1, slots, stride_group=g)
        ev = sim(slots)
        y, fo = LY.conv2d(ev, LY.SimCt(LY.pack(X, fm, slots), 22), fm, 32, 3, 2, 1, kern, masks, slots,
                          stride_group=g)
        out.append((ev.ks, y, fo))
    assert out[0][0] == 549 and out[1][0] == 579
    assert np.array_equal(out[0][1].v, out[1][1].v) and out[1][1].level == out[0][1].level == 17
    assert np.max(np.abs(LY.unpack(out[1][1].v, out[1][2]) - LY.conv2d_ref(X, K, 2, 1))) < 1e-12
    assert len(LY.conv_rotations(fm, 32, 3, 2, 1, slots, stride_group=16)) == len(
        LY.conv_rotations(fm, 32, 3, 2, 1, slots)) + 1


@pytest.mark.parametrize("C,F,HW,k,S,P", [(3, 4, 12, 3, 2, 1), (2, 2, 13, 5, 2, 2), (1, 2, 16, 3, 3, 0)])
def test_sim_conv_log_step_striding(C, F, HW, k, S, P):
    slots = 4096
    X = synth.image(17, C, HW, HW)
    K = synth.conv_weights(17, F, C, k, 0.2)
    fm = LY.FMap(C, HW, HW)
    kern, masks = LY.conv_plaintexts(fm, K, S, P, slots, stride_log=True)
    ev = sim(slots)
    y, fo = LY.conv2d(ev, LY.SimCt(LY.pack(X, fm, slots), 12), fm, F, k, S, P, kern, masks, slots, stride_log=True)
    assert fo == LY.conv_out_map(fm, F, k, S, P, slots)
    assert np.max(np.abs(LY.unpack(y.v, fo) - LY.conv2d_ref(X, K, S, P))) < 1e-12
    assert set(LY.conv_rotations(fm, F, k, S, P, slots, stride_log=True)) >= {(S - 1) << t for t in range(
        LY.log_steps(fo.W))}


def test_sim_pool_log_step_striding():
    slots = 8192
    X = synth.image(18, 6, 24, 24)
    fm = LY.FMap(6, 24, 24, 28, 784)
    ev = sim(slots)
    pm = LY.avgpool_plaintexts(fm, 2, 2, slots, stride_log=True)
    z, f2 = LY.avgpool(ev, LY.SimCt(LY.pack(X, fm, slots), 5), fm, 2, 2, pm, stride_log=True)
    assert f2 == LY.FMap(6, 12, 12) and ev.ks == 3 + 4 + 11 + 5 and z.level == 5 - 6
    assert np.max(np.abs(LY.unpack(z.v, f2) - LY.avgpool_ref(X, 2, 2))) < 1e-12


def test_padding_beyond_half_kernel_takes_the_relayout():
    assert LY.conv_kind(3, 2) == "padded" and LY.conv_kind(5, 3, LY.FMap(1, 8, 8)) == "padded"
    assert LY.conv_kind(1, 1) == "padded" and LY.conv_kind(5, 2) == "generic"
    with pytest.raises(ValueError):
        LY.conv_kind(3, -1)
    with pytest.raises(ValueError):  # 4 padded 16 x 16 blocks (20 x 20 each) exceed 1024 slots
        LY.pad_masks(LY.FMap(4, 16, 16), 2, 1024)


PAD_MAPS = [  # (C, H, W, rs, cs, P)
    (1, 6, 6, None, None, 2),
    (3, 5, 7, None, None, 3),    # rectangular
    (4, 8, 8, None, None, 1),
    (2, 6, 6, 16, 96, 2),        # wide rows: channels spread first
    (2, 6, 6, 30, 180, 2),       # rows too wide for the padded block: rows first
    (2, 4, 4, 8, 64, 2),         # rows already at W + 2P and cs = H_p W_p: a clearing mask only
]


@pytest.mark.parametrize("C,H,W,rs,cs,P", PAD_MAPS)
@pytest.mark.parametrize("bsgs", [False, True], ids=["horner", "bsgs"])
def test_pad_layout_builds_the_padded_tensor(C, H, W, rs, cs, P, bsgs):
    """The re-layout yields exactly np.pad(X) flattened in X_p's map, zero
    in every other slot, even when the unused input slots hold junk; it uses
    the three keys and the level count pad_plan states."""
    slots = 2048
    X = synth.image(31, C, H, W)
    fm = LY.FMap(C, H, W, rs, cs)
    v = LY.pack(X, fm, slots)
    used = LY.pack(np.ones_like(X), fm, slots) != 0
    junk = np.random.default_rng(5).uniform(-3, 3, slots)
    v[~used] = junk[~used]
    masks = LY.pad_masks(fm, P, slots, bsgs)
    ev = sim(slots)
    xp, fp = LY.pad_layout(ev, LY.SimCt(v, 5), fm, P, masks, bsgs)
    assert fp == LY.FMap(C, H + 2 * P, W + 2 * P)
    want = np.zeros(slots)
    want[:C * fp.cs] = np.pad(X, ((0, 0), (P, P), (P, P))).reshape(-1)
    assert np.array_equal(xp.v, want)
    steps, shift, _ = LY.pad_plan(fm, P)
    assert shift == -(P * (W + 2 * P) + P)
    assert xp.level == 5 - len(steps)
    assert ev.ks == 1 + sum(LY.masked_chain_switches(n, bsgs) for _, n, _ in steps)
    assert len(LY.pad_keys(fm, P)) <= 3
    if rs is None:  # dense input: channels spread first, then rows
        assert [s[0] for s in steps] == (["chan", "row"] if C > 1 else ["row"])
        assert ev.ks == 1 + (C - 1) + (H - 1) if not bsgs else True
    if rs == 30:
        assert [s[0] for s in steps] == ["row", "chan"]
    if rs == 8:
        assert steps == [("clear", 1, 0)]


@pytest.mark.parametrize("C,F,H,W,k,S,P", [
    (2, 3, 8, 8, 3, 1, 2),     # 3x3 with padding 2 (output wider than the input)
    (3, 2, 10, 10, 1, 2, 1),   # 1x1 / stride 2 / padding 1 (ResNet downsampling shortcut)
    (1, 1, 6, 6, 3, 1, 3),
    (2, 2, 7, 9, 5, 2, 3),     # rectangular, strided
    (4, 1, 5, 5, 3, 1, 2),
])
def test_sim_padded_conv(C, F, H, W, k, S, P):
    """Padding beyond (k-1)/2: re-layout then the generic P = 0 schedule
    equals the FP64 convolution with padding P."""
    slots = 4096
    X = synth.image(33, C, H, W)
    K = synth.conv_weights(33, F, C, k, 0.2)
    fm = LY.FMap(C, H, W)
    assert LY.conv_kind(k, P, fm, F) == "padded"
    kern, masks = LY.conv_plaintexts(fm, K, S, P, slots)
    ev = sim(slots)
    y, fo = LY.conv2d(ev, LY.SimCt(LY.pack(X, fm, slots), 12), fm, F, k, S, P, kern, masks, slots)
    Ho, Wo = (H + 2 * P - k) // S + 1, (W + 2 * P - k) // S + 1
    assert (fo.C, fo.H, fo.W) == (F, Ho, Wo) and fo == LY.conv_out_map(fm, F, k, S, P, slots)
    assert np.max(np.abs(LY.unpack(y.v, fo) - LY.conv2d_ref(X, K, S, P))) < 1e-12
    fp = LY.padded_map(fm, P)
    keys = set(LY.conv_rotations(fm, F, k, S, P, slots))
    assert keys == LY.pad_keys(fm, P) | set(LY.conv_rotations(fp, F, k, S, 0, slots))
    assert {i * fp.rs + j for i in range(k) for j in range(k)} - {0} <= keys


# ------------------------------------------------------------------ encrypted (oracle CKKS)
def he_eval(name, rots, relin=False):
    ctx, sk, pk = H.oracle_ctx(name)
    keys = H.oracle_keys(name, rots)
    return LY.HEEval(ctx, keys, H.oracle_key(name, "relin") if relin else None), ctx, sk, pk


def encode_all(ctx, vecs, level):
    return [ctx.encode(v, ctx.pr.scale, level) for v in vecs]


def test_he_config0_conv_decrypts_to_fp64():
    name = "config0"
    ctx0, _, _ = H.oracle_ctx(name)
    slots = ctx0.n // 2
    X = synth.image(10, 1, 8, 8)
    K = synth.conv_weights(10, 1, 1, 3, 0.1)
    fm = LY.FMap(1, 8, 8)
    ev, ctx, sk, pk = he_eval(name, LY.conv_rotations(fm, 1, 3, 1, 1, slots))
    kern, masks = LY.conv_plaintexts(fm, K, 1, 1, slots)
    _, ct = H.encrypt_slots(name, 10, values=LY.pack(X, fm, slots))
    y, fo = LY.conv2d(ev, ct, fm, 1, 3, 1, 1, encode_all(ctx, kern, ctx.pr.L), masks, slots)
    assert ev.ks == 8
    err = np.max(np.abs(LY.unpack(ctx.decrypt(sk, y), fo) - LY.conv2d_ref(X, K, 1, 1)))
    assert err < 1e-3, err


def test_he_config1_stack_decrypts_to_fp64():
    name = "config1"
    ctx1, _, _ = H.oracle_ctx(name)
    slots = ctx1.n // 2
    X = synth.image(11, 1, 28, 28)
    K = synth.conv_weights(11, 6, 1, 5, 0.1)
    fm = LY.FMap(1, 28, 28)
    f1 = LY.conv_out_map(fm, 6, 5, 1, 0, slots)
    rots = sorted(set(LY.conv_rotations(fm, 6, 5, 1, 0, slots)) | set(LY.avgpool_rotations(f1, 2, 2)))
    ev, ctx, sk, pk = he_eval(name, rots, relin=True)
    kern, masks = LY.conv_plaintexts(fm, K, 1, 0, slots)
    _, ct = H.encrypt_slots(name, 11, values=LY.pack(X, fm, slots))
    L = ctx.pr.L
    y, f1 = LY.conv2d(ev, ct, fm, 6, 5, 1, 0, encode_all(ctx, kern, L), masks, slots)
    p = LY.relu_poly4(ev, y, ctx.pr.scale)
    z, f2 = LY.avgpool(ev, p, f1, 2, 2, encode_all(ctx, LY.avgpool_plaintexts(f1, 2, 2, slots), L))
    assert z.level == 1 and ev.ks == 61
    ref = LY.avgpool_ref(LY.relu4_ref(LY.conv2d_ref(X, K, 1, 0)), 2, 2)
    err = np.max(np.abs(LY.unpack(ctx.decrypt(sk, z), f2) - ref))
    assert err < 1e-2, err


def test_he_config1_padded_conv_decrypts():
    """7x7 / stride 2 / padding 3 on 3 x 16 x 16 (C=3 -> F=2) at N=2^14."""
    name = "config1"
    ctx1, _, _ = H.oracle_ctx(name)
    slots = ctx1.n // 2
    X = synth.image(12, 3, 16, 16)
    K = synth.conv_weights(12, 2, 3, 7, 0.1)
    fm = LY.FMap(3, 16, 16)
    ev, ctx, sk, pk = he_eval(name, LY.conv_rotations(fm, 2, 7, 2, 3, slots))
    kern, masks = LY.conv_plaintexts(fm, K, 2, 3, slots)
    _, ct = H.encrypt_slots(name, 12, values=LY.pack(X, fm, slots))
    L = ctx.pr.L
    y, fo = LY.conv2d(ev, ct, fm, 2, 7, 2, 3, encode_all(ctx, kern, L), encode_all(ctx, masks, L - 1), slots)
    err = np.max(np.abs(LY.unpack(ctx.decrypt(sk, y), fo) - LY.conv2d_ref(X, K, 2, 3)))
    assert err < 1e-3, err


def test_he_config1_relayout_padded_conv_decrypts():
    """3x3 / padding 2 on 2 x 6 x 6 (C=2 -> F=2) at N=2^14: re-layout (two
    mask levels) then the generic schedule."""
    name = "config1"
    ctx1, _, _ = H.oracle_ctx(name)
    slots = ctx1.n // 2
    X = synth.image(13, 2, 6, 6)
    K = synth.conv_weights(13, 2, 2, 3, 0.2)
    fm = LY.FMap(2, 6, 6)
    ev, ctx, sk, pk = he_eval(name, LY.conv_rotations(fm, 2, 3, 1, 2, slots))
    kern, masks = LY.conv_plaintexts(fm, K, 1, 2, slots)
    npad = len(LY.pad_masks(fm, 2, slots))
    _, ct = H.encrypt_slots(name, 13, values=LY.pack(X, fm, slots))
    L = ctx.pr.L
    steps, _, _ = LY.pad_plan(fm, 2)
    assert [(st, n) for st, n, _ in steps] == [("chan", 2), ("row", 6)] and npad == 8
    pm = encode_all(ctx, masks[:2], L) + encode_all(ctx, masks[2:npad], L - 1)
    y, fo = LY.conv2d(ev, ct, fm, 2, 3, 1, 2, encode_all(ctx, kern, L - 2), pm + encode_all(ctx, masks[npad:], L - 3), slots)
    assert y.level == L - 4
    err = np.max(np.abs(LY.unpack(ctx.decrypt(sk, y), fo) - LY.conv2d_ref(X, K, 1, 2)))
    assert err < 1e-3, err


def test_he_config1_log_step_strided_conv_decrypts():
    """3x3 / stride 2 / padding 1 on 3 x 12 x 12 -> 4 x 6 x 6 with striding
    approach 2 at N=2^14."""
    name = "config1"
    ctx1, _, _ = H.oracle_ctx(name)
    slots = ctx1.n // 2
    X = synth.image(14, 3, 12, 12)
    K = synth.conv_weights(14, 4, 3, 3, 0.2)
    fm = LY.FMap(3, 12, 12)
    ev, ctx, sk, pk = he_eval(name, LY.conv_rotations(fm, 4, 3, 2, 1, slots, stride_log=True))
    kern, masks = LY.conv_plaintexts(fm, K, 2, 1, slots, stride_log=True)
    _, ct = H.encrypt_slots(name, 14, values=LY.pack(X, fm, slots))
    L = ctx.pr.L
    y, fo = LY.conv2d(ev, ct, fm, 4, 3, 2, 1, encode_all(ctx, kern, L), encode_all(ctx, masks, L), slots,
                      stride_log=True)
    assert fo == LY.FMap(4, 6, 6) and y.level == L - 7  # kernel, block mask, 3 log steps, rows, channels
    err = np.max(np.abs(LY.unpack(ctx.decrypt(sk, y), fo) - LY.conv2d_ref(X, K, 2, 1)))
    assert err < 1e-3, err


@pytest.mark.slow
def test_he_config2_small_special_conv_decrypts():
    """Special convolution at the N=2^16, L=24 parameters with 4 replicated
    channels of 64x64 (2*C*W^2 = N/2): 20 key switches."""
    name = "config2"
    ctx2, _, _ = H.oracle_ctx(name)
    slots = ctx2.n // 2
    X = synth.image(12, 4, 64, 64)
    K = synth.conv_weights(12, 4, 4, 3, (2.0 / 36) ** 0.5)
    fm = LY.FMap(4, 64, 64, reps=2)
    ev, ctx, sk, pk = he_eval(name, LY.conv_rotations(fm, 4, 3, 1, 1, slots))
    kern, masks = LY.conv_plaintexts(fm, K, 1, 1, slots)
    _, ct = H.encrypt_slots(name, 12, values=LY.pack(X, fm, slots))
    L = ctx.pr.L
    y, fo = LY.conv2d(ev, ct, fm, 4, 3, 1, 1, encode_all(ctx, kern, L), encode_all(ctx, masks, L), slots)
    assert ev.ks == 20
    err = np.max(np.abs(LY.unpack(ctx.decrypt(sk, y), fo) - LY.conv2d_ref(X, K, 1, 1)))
    assert err < 1e-3, err


# ---------------------------------------------------------------- log-step channel sum
def test_channel_sum_keys_closed_form():
    assert LY.channel_sum_keys(16, 1024, True) == {1024, 2048, 4096, 8192}
    assert LY.channel_sum_keys(16, 1024, False) == {1024}
    assert LY.channel_sum_keys(6, 784, True) == {784}  # not a power of two: the chain
    assert LY.channel_sum_keys(1, 784, True) == set()
    assert LY.channel_sum_keys(2, 5, True) == {5}


@pytest.mark.parametrize("C", [2, 4, 8, 16])
def test_channel_sum_logstep_equals_chain_and_brute_force(C):
    """Doubling and the chain give the same slot vector, and it equals the sum
    of the C cyclic shifts written out (rotation = left shift of the slots)."""
    slots = 4096
    step = 37
    rng = np.random.default_rng(C)
    v = rng.uniform(-1, 1, slots)
    want = sum(np.roll(v, -j * step) for j in range(C))
    for logstep, ks in ((False, C - 1), (True, C.bit_length() - 1)):
        ev = sim(slots)
        S = LY.channel_sum(ev, LY.SimCt(v, 3), C, step, logstep)
        assert ev.ks == ks
        assert np.max(np.abs(S.v - want)) < 1e-12


@pytest.mark.parametrize("stride,F", [(1, 16), (2, 32)])
def test_sim_config2_special_conv_logstep(stride, F):
    """The ResNet-shaped special convolutions with the log-step channel sum:
    same output as the FP64 convolution with F log2(C) instead of F (C - 1)
    channel-sum key switches."""
    slots = 32768
    X = synth.image(2, 16, 32, 32)
    K = synth.conv_weights(2, F, 16, 3, (2.0 / 144) ** 0.5)
    fm = LY.FMap(16, 32, 32, reps=2)
    kern, masks = LY.conv_plaintexts(fm, K, stride, 1, slots)
    ev = sim(slots)
    y, fo = LY.conv2d(ev, LY.SimCt(LY.pack(X, fm, slots), 24), fm, F, 3, stride, 1, kern, masks, slots,
                      logstep=True)
    assert np.max(np.abs(LY.unpack(y.v, fo) - LY.conv2d_ref(X, K, stride, 1))) < 1e-9
    if stride == 1:
        assert ev.ks == 8 + 16 * 4 and np.array_equal(y.v[:16384], y.v[16384:])
    else:
        assert ev.ks == 549 - 32 * 15 + 32 * 4
    keys = LY.conv_rotations(fm, F, 3, stride, 1, slots, logstep=True)
    assert {1024, 2048, 4096, 8192} <= set(keys) and len(keys) == (8 if stride == 1 else 10)


def test_sim_generic_conv_logstep():
    """Generic convolution (5x5, pad 2, stride 2) over 4 input channels with
    the log-step channel sum: equals the FP64 convolution."""
    slots = 8192
    X = synth.image(5, 4, 16, 16)
    K = synth.conv_weights(5, 3, 4, 5, 0.1)
    fm = LY.FMap(4, 16, 16)
    kern, masks = LY.conv_plaintexts(fm, K, 2, 2, slots)
    ev = sim(slots)
    y, fo = LY.conv2d(ev, LY.SimCt(LY.pack(X, fm, slots), 12), fm, 3, 5, 2, 2, kern, masks, slots, logstep=True)
    assert np.max(np.abs(LY.unpack(y.v, fo) - LY.conv2d_ref(X, K, 2, 2))) < 1e-9
    chain = sim(slots)
    LY.conv2d(chain, LY.SimCt(LY.pack(X, fm, slots), 12), fm, 3, 5, 2, 2, kern, masks, slots)
    assert chain.ks - ev.ks == 3 * (3 - 2)


@pytest.mark.slow
def test_he_config2_small_special_conv_logstep_decrypts():
    """The encrypted special convolution with the log-step channel sum (4
    replicated channels of 64x64 at N=2^16): 8 + 4 * 2 key switches."""
    name = "config2"
    ctx2, _, _ = H.oracle_ctx(name)
    slots = ctx2.n // 2
    X = synth.image(12, 4, 64, 64)
    K = synth.conv_weights(12, 4, 4, 3, (2.0 / 36) ** 0.5)
    fm = LY.FMap(4, 64, 64, reps=2)
    ev, ctx, sk, pk = he_eval(name, LY.conv_rotations(fm, 4, 3, 1, 1, slots, logstep=True))
    kern, masks = LY.conv_plaintexts(fm, K, 1, 1, slots)
    _, ct = H.encrypt_slots(name, 12, values=LY.pack(X, fm, slots))
    L = ctx.pr.L
    y, fo = LY.conv2d(ev, ct, fm, 4, 3, 1, 1, encode_all(ctx, kern, L), encode_all(ctx, masks, L), slots,
                      logstep=True)
    assert ev.ks == 16
    err = np.max(np.abs(LY.unpack(ctx.decrypt(sk, y), fo) - LY.conv2d_ref(X, K, 1, 1)))
    assert err < 1e-3, err


# ---------------------------------------------------------------- baby-step giant-step masked chains
def test_bsgs_split_closed_form():
    assert [LY.bsgs_split(n) for n in (1, 2, 3, 4, 5, 6, 12, 16, 17, 32)] == [
        (1, 1), (2, 1), (2, 2), (2, 2), (3, 2), (3, 2), (4, 3), (4, 4), (5, 4), (6, 6)]
    assert LY.masked_chain_switches(32, True) == 10 and LY.masked_chain_switches(32, False) == 31
    assert LY.masked_chain_keys(16, 48, True) == {48, 96, 144, 192}
    assert LY.masked_chain_keys(16, 48, False) == {48} and LY.masked_chain_keys(1, 48, True) == set()


@pytest.mark.parametrize("n,key", [(1, 5), (2, -1), (5, 7), (12, 255), (16, 1), (17, -33), (32, 768)])
def test_masked_chain_bsgs_brute_force(n, key):
    """sum_t Rot_{t key}(v m_t) written out with np.roll, against the Horner
    chain (plain masks) and the baby-step giant-step chain (pre-rotated masks)."""
    slots = 2048
    rng = np.random.default_rng(n * 1000 + abs(key))
    v = rng.uniform(-1, 1, slots)
    ms = [rng.uniform(-1, 1, slots) for _ in range(n)]
    want = sum(np.roll(v * m, -t * key) for t, m in enumerate(ms))
    for bsgs in (False, True):
        ev = sim(slots)
        got = LY.masked_chain(ev, LY.SimCt(v, 4), LY.chain_masks(ms, key, bsgs), n, key, bsgs)
        assert ev.ks == LY.masked_chain_switches(n, bsgs) and got.level == 3
        assert np.max(np.abs(got.v - want)) < 1e-12


def test_sim_config2_conv_b_logstep_bsgs():
    """Conv B (16 -> 32, stride 2) with both options: 8 + 32 * 4 + (6 + 6 + 10)
    key switches instead of 549, same output as the FP64 convolution."""
    slots = 32768
    X = synth.image(2, 16, 32, 32)
    K = synth.conv_weights(2, 32, 16, 3, (2.0 / 144) ** 0.5)
    fm = LY.FMap(16, 32, 32, reps=2)
    kern, masks = LY.conv_plaintexts(fm, K, 2, 1, slots, bsgs=True)
    ev = sim(slots)
    y, fo = LY.conv2d(ev, LY.SimCt(LY.pack(X, fm, slots), 24), fm, 32, 3, 2, 1, kern, masks, slots,
                      logstep=True, bsgs=True)
    assert np.max(np.abs(LY.unpack(y.v, fo) - LY.conv2d_ref(X, K, 2, 1))) < 1e-9
    assert ev.ks == 8 + 32 * 4 + 22 and 24 - y.level == 5 and fo == LY.FMap(32, 16, 16)
    # taps {+-W, +-1}, column chain {1, 2, 3, 4} (1 shared with a tap), row chain
    # 48 {1..4}, channel chain 768 {1..6}, channel sum 1024 {1, 2, 4, 8}
    assert len(LY.conv_rotations(fm, 32, 3, 2, 1, slots, logstep=True, bsgs=True)) == 4 + 3 + 4 + 6 + 4


@pytest.mark.parametrize("C,HW,ks", [(32, 16, 8 + 10), (64, 8, 6 + 14)])
def test_sim_gap_bsgs(C, HW, ks):
    slots = 32768
    X = synth.image(4, C, HW, HW)
    fm = LY.FMap(C, HW, HW)
    ev = sim(slots)
    y, fo = LY.gap(ev, LY.SimCt(LY.pack(X, fm, slots), 10), fm, LY.gap_plaintexts(fm, slots, bsgs=True), bsgs=True)
    assert ev.ks == ks and y.level == 9
    assert np.max(np.abs(y.v[:C] - LY.gap_ref(X))) < 1e-12 and np.max(np.abs(y.v[C:])) < 1e-12


def test_he_config1_stack_bsgs_decrypts_to_fp64():
    """The LeNet-shaped stack with the baby-step giant-step compaction in the
    average pool: 61 - 27 + 13 key switches, decrypts to the FP64 layers."""
    name = "config1"
    ctx1, _, _ = H.oracle_ctx(name)
    slots = ctx1.n // 2
    X = synth.image(11, 1, 28, 28)
    K = synth.conv_weights(11, 6, 1, 5, 0.1)
    fm = LY.FMap(1, 28, 28)
    f1 = LY.conv_out_map(fm, 6, 5, 1, 0, slots)
    rots = sorted(set(LY.conv_rotations(fm, 6, 5, 1, 0, slots, bsgs=True)) |
                  set(LY.avgpool_rotations(f1, 2, 2, bsgs=True)))
    ev, ctx, sk, pk = he_eval(name, rots, relin=True)
    kern, masks = LY.conv_plaintexts(fm, K, 1, 0, slots, bsgs=True)
    _, ct = H.encrypt_slots(name, 11, values=LY.pack(X, fm, slots))
    L = ctx.pr.L
    y, f1 = LY.conv2d(ev, ct, fm, 6, 5, 1, 0, encode_all(ctx, kern, L), masks, slots, bsgs=True)
    p = LY.relu_poly4(ev, y, ctx.pr.scale)
    z, f2 = LY.avgpool(ev, p, f1, 2, 2, encode_all(ctx, LY.avgpool_plaintexts(f1, 2, 2, slots, bsgs=True), L),
                       bsgs=True)
    assert z.level == 1 and ev.ks == 61 - 27 + 13
    ref = LY.avgpool_ref(LY.relu4_ref(LY.conv2d_ref(X, K, 1, 0)), 2, 2)
    err = np.max(np.abs(LY.unpack(ctx.decrypt(sk, z), f2) - ref))
    assert err < 1e-2, err


# ---------------------------------------------------------------- diagonal fully connected layer
@pytest.mark.parametrize("n_in,n_out", [(64, 10), (32, 32), (16, 1), (8, 5), (2, 2)])
def test_sim_fc_diag(n_in, n_out):
    """Halevi-Shoup diagonal form with baby-step giant-step: equals the FP64
    matrix-vector product written out; 1 + (B-1) + (A-1) key switches, one
    level, zeros outside the n_out outputs."""
    slots = 4096
    x = synth.uniform_slots(9 + n_in, n_in)
    Wm = synth.fc_weights(9 + n_out, n_out, n_in, (2.0 / n_in) ** 0.5)
    v = np.zeros(slots)
    v[:n_in] = x
    diags = LY.fc_diag_plaintexts(Wm, slots)
    ev = sim(slots)
    y = LY.fc_diag(ev, LY.SimCt(v, 5), n_in, n_out, diags)
    B, A = LY.bsgs_split(n_in)
    assert ev.ks == 1 + (B - 1) + (A - 1) and y.level == 4
    want = np.array([sum(Wm[j][i] * x[i] for i in range(n_in)) for j in range(n_out)])
    assert np.max(np.abs(y.v[:n_out] - want)) < 1e-12 and np.max(np.abs(y.v[n_out:])) < 1e-12
    assert LY.fc_diag_rotations(n_in) == sorted({-n_in} | set(range(1, B)) | ({B} if A > 1 else set()))


def test_sim_fc_diag_resnet_shape_key_switches():
    """The ResNet-shaped FC 64 -> 10: 15 key switches and one level instead of 69 and two."""
    slots = 32768
    x = synth.uniform_slots(5, 64)
    Wm = synth.fc_weights(5, 10, 64, (2.0 / 64) ** 0.5)
    v = np.zeros(slots)
    v[:64] = x
    ev = sim(slots)
    y = LY.fc_diag(ev, LY.SimCt(v, 10), 64, 10, LY.fc_diag_plaintexts(Wm, slots))
    assert ev.ks == 15 and y.level == 9
    assert np.max(np.abs(y.v[:10] - LY.fc_ref(x, Wm))) < 1e-12


def test_he_config1_fc_diag_decrypts():
    """Encrypted diagonal FC 64 -> 10 at N=2^14 decrypts to W x within 1e-3."""
    name = "config1"
    ctx1, _, _ = H.oracle_ctx(name)
    slots = ctx1.n // 2
    x = synth.uniform_slots(77, 64)
    Wm = synth.fc_weights(77, 10, 64, (2.0 / 64) ** 0.5)
    v = np.zeros(slots)
    v[:64] = x
    ev, ctx, sk, pk = he_eval(name, LY.fc_diag_rotations(64))
    _, ct = H.encrypt_slots(name, 77, values=v)
    y = LY.fc_diag(ev, ct, 64, 10, encode_all(ctx, LY.fc_diag_plaintexts(Wm, slots), ctx.pr.L))
    assert ev.ks == 15 and y.level == ctx.pr.L - 1
    err = np.max(np.abs(ctx.decrypt(sk, y)[:10] - LY.fc_ref(x, Wm)))
    assert err < 1e-3, err
