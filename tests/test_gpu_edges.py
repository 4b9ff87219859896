"""Edge and degenerate cases against the oracle (needs MI355X)."""
import numpy as np
import pytest
import torch

import synth
from oracle import ckks
from oracle import layers as LY
from tests import helpers as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g1():
    g = H.gpu_ctx("config1")
    yield g
    g.close()


def test_keyswitch_at_level_one(g1):
    """One limb left: a single one-limb digit, basis extension to P only."""
    name = "config1"
    octx, _, _ = H.oracle_ctx(name)
    for r in (1, -5):
        g1.key_upload(r, H.oracle_key(name, r))
    _, a = H.encrypt_slots(name, 60, level=1)
    got = g1.rotate_hoisted(g1.ct_from_numpy(a.data, a.scale, cap=8), [1, -5])
    want = octx.rotate_hoisted(a, [1, -5], H.oracle_keys(name, [1, -5]))
    for x, y in zip(got, want):
        H.assert_limbs_equal(x.numpy(), y.data, "level-1 rotation")
    from paper_2510_03996_amd import he

    g1.key_upload(he.KEY_RELIN, H.oracle_key(name, "relin"))
    _, b = H.encrypt_slots(name, 61, level=1, enc_id=1)
    m = g1.mul_relin(g1.ct_from_numpy(a.data, a.scale), g1.ct_from_numpy(b.data, b.scale))
    H.assert_limbs_equal(m.numpy(), octx.mul_relin(a, b, H.oracle_key(name, "relin")).data, "level-1 relin")


def test_degenerate_rotation_sets(g1):
    name = "config1"
    octx, _, _ = H.oracle_ctx(name)
    n2 = octx.n // 2
    g1.key_upload(3, H.oracle_key(name, 3))
    _, a = H.encrypt_slots(name, 62)
    ga = g1.ct_from_numpy(a.data, a.scale)
    assert g1.rotate_hoisted(ga, [], outs=[]) == []
    # rotations by 0 and by N/2 are copies and need no key
    for r in (0, n2, -n2):
        H.assert_limbs_equal(g1.rotate(ga, r).numpy(), a.data, "rotation by %d" % r)
    # amounts equal mod N/2 share one key and one result
    want = octx.rotate(a, 3, {3: H.oracle_key(name, 3)})
    outs = g1.rotate_hoisted(ga, [3, 3 - n2, 3 + n2, 0])
    for o in outs[:3]:
        H.assert_limbs_equal(o.numpy(), want.data, "rotation aliases")
    H.assert_limbs_equal(outs[3].numpy(), a.data, "copy in a hoisted set")
    # two outputs in one buffer are rejected (they may be written from different streams)
    from paper_2510_03996_amd import he

    o = g1.new_ct(a.level)
    with pytest.raises(he.HEError) as e:
        g1.rotate_hoisted(ga, [3, 0], outs=[o, o])
    assert e.value.name == "HE_EINVAL"


def test_constants_and_rescale_chain(g1):
    name = "config1"
    octx, sk, _ = H.oracle_ctx(name)
    v, a = H.encrypt_slots(name, 63)
    ga = g1.ct_from_numpy(a.data, a.scale)
    sc = octx.pr.scale
    for c in (-0.37, 0.0, 1.0, -2.5):
        got = g1.mul_const(ga, c, sc)
        want = octx.mul_plain(a, octx.encode_const(c, sc, a.level))
        H.assert_limbs_equal(got.numpy(), want.data, "mul_const %g" % c)
        got2 = g1.add_const(ga, c)
        want2 = octx.add_plain(a, octx.encode_const(c, a.scale, a.level))
        H.assert_limbs_equal(got2.numpy(), want2.data, "add_const %g" % c)
    # rescale all the way down to level 1
    x, ox = g1.mul_const(ga, 0.5, sc), octx.mul_plain(a, octx.encode_const(0.5, sc, a.level))
    while ox.level > 1:
        x, ox = g1.rescale(x), octx.rescale(ox)
        H.assert_limbs_equal(x.numpy(), ox.data, "rescale to level %d" % ox.level)
        assert x.scale == ox.scale
        if ox.level > 1:
            x, ox = g1.mul_const(x, 1.0, sc), octx.mul_plain(ox, octx.encode_const(1.0, sc, ox.level))
    assert np.max(np.abs(octx.decrypt(sk, ckks.Ciphertext(x.numpy(), x.scale)) - 0.5 * v)) < 1e-3


def test_fc_single_output_with_bias_and_stride1_pool(g1):
    name = "config1"
    octx, sk, _ = H.oracle_ctx(name)
    slots = octx.n // 2
    x = synth.uniform_slots(64, 16)
    Wm = synth.fc_weights(64, 1, 16, 0.3)
    plan = g1.fc_plan(16, 1)
    assert -1 not in plan.keys()
    for r in plan.keys():
        g1.key_upload(r, H.oracle_key(name, r))
    v = np.zeros(slots)
    v[:16] = x
    _, ct = H.encrypt_slots(name, 64, values=v)
    rows, masks = LY.fc_plaintexts(Wm, slots)
    rp = [octx.encode(r, octx.pr.scale, ct.level) for r in rows]
    mp = [octx.encode(m, octx.pr.scale, ct.level) for m in masks]
    ev = LY.HEEval(octx, H.oracle_keys(name, plan.keys()))
    want = LY.fc(ev, ct, 16, 1, rp, mp)
    bias = octx.encode(np.full(slots, 0.25), want.scale, want.level)
    want = octx.add_plain(want, bias)
    got = g1.fc(g1.ct_from_numpy(ct.data, ct.scale), 16, 1, [g1.pt_from_numpy(p.data, p.scale) for p in rp],
                [g1.pt_from_numpy(p.data, p.scale) for p in mp], bias_pt=g1.pt_from_numpy(bias.data, bias.scale))
    H.assert_limbs_equal(got.numpy(), want.data, "fc 16->1 + bias")
    dec = octx.decrypt(sk, ckks.Ciphertext(got.numpy(), got.scale))
    assert abs(dec[0] - (Wm[0] @ x + 0.25)) < 1e-3
    # stride-1 average pooling (one 1/k^2 mask, no compaction)
    X = synth.image(65, 2, 6, 6)
    fm = LY.FMap(2, 6, 6)
    pl = g1.avgpool_plan(LY_to_he(fm), 2, 1)
    for r in pl.keys():
        g1.key_upload(r, H.oracle_key(name, r))
    _, cx = H.encrypt_slots(name, 65, values=LY.pack(X, fm, slots))
    mpts = [octx.encode(m, octx.pr.scale, cx.level) for m in LY.avgpool_plaintexts(fm, 2, 1, slots)]
    ev = LY.HEEval(octx, H.oracle_keys(name, pl.keys()))
    want, fo = LY.avgpool(ev, cx, fm, 2, 1, mpts)
    got, gfo = g1.avgpool(g1.ct_from_numpy(cx.data, cx.scale), LY_to_he(fm), 2, 1,
                          [g1.pt_from_numpy(p.data, p.scale) for p in mpts])
    assert gfo.key() == fo.key()
    H.assert_limbs_equal(got.numpy(), want.data, "stride-1 avgpool")
    dec = LY.unpack(octx.decrypt(sk, ckks.Ciphertext(got.numpy(), got.scale)), fo)
    assert np.max(np.abs(dec - LY.avgpool_ref(X, 2, 1))) < 1e-3


def LY_to_he(fm):
    from paper_2510_03996_amd import he

    return he.he_fmap(*fm.key())


def test_minimal_batch(g1):
    from paper_2510_03996_amd import he

    name = "config1"
    octx, _, _ = H.oracle_ctx(name)
    g1.key_upload(7, H.oracle_key(name, 7))
    _, a = H.encrypt_slots(name, 66)
    pt = octx.encode(synth.uniform_slots(66, octx.n // 2, stream=9), octx.pr.scale, a.level)
    inp = he.to_device(a.data[None])
    pool = he.to_device(pt.data[None])
    out = torch.zeros((1, 2, a.level - 1, octx.n), dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    b = he.Batch(g1, inp, a.level, a.scale, [[7]], [1], pool, pt.scale, [[0]], out, he.BATCH_GRAPH | he.BATCH_TUNE)
    with torch.cuda.stream(s):
        b.run(s)
        s.synchronize()
    want = octx.rescale(octx.mul_plain(octx.rotate(a, 7, {7: H.oracle_key(name, 7)}), pt))
    H.assert_limbs_equal(out[0].cpu().numpy().view(np.uint64), want.data, "one-item batch")
    b.close()


def test_argument_errors(g1):
    from paper_2510_03996_amd import he

    with pytest.raises(he.HEError) as e:
        he.Context(13, [40, 40], [41], 1)
    assert e.value.name == "HE_EINVAL"
    with pytest.raises(he.HEError) as e:
        he.Context(14, [40] * 12, [41] * 11, 11)  # more than ten limbs per basis conversion
    assert e.value.name == "HE_EINVAL"
    with pytest.raises(he.HEError) as e:
        g1.key_upload(11, np.zeros(10, dtype=np.uint64))
    assert e.value.name == "HE_EINVAL"
    _, a = H.encrypt_slots("config1", 67)
    ga = g1.ct_from_numpy(a.data, a.scale)
    small = g1.new_ct(2)
    with pytest.raises(he.HEError) as e:
        g1.add(ga, ga, out=small)
    assert e.value.name == "HE_EINVAL"
    with pytest.raises(he.HEError) as e:
        g1.key_evict(12345)
    assert e.value.name == "HE_ENOKEY"


def test_product_sum_and_monomial_errors(g1):
    """he_mac_plain, he_mul_i and he_mod_raise reject mismatched inputs
    before any work; a one-term product sum equals he_mul_plain; ±i in place
    and a raise to level 1 (a copy of limb 0) against the oracle."""
    from oracle import boot as BT
    from paper_2510_03996_amd import he

    name = "config1"
    octx, _, _ = H.oracle_ctx(name)
    _, a = H.encrypt_slots(name, 80, enc_id=0)
    _, b = H.encrypt_slots(name, 81, level=5, enc_id=1)
    _, p = H.encode_slots(name, 82, octx.pr.L)
    ga, gb = g1.ct_from_numpy(a.data, a.scale), g1.ct_from_numpy(b.data, b.scale)
    gp = g1.pt_from_numpy(p.data, p.scale)
    one = g1.mac_plain([ga], [gp])
    H.assert_limbs_equal(one.numpy(), octx.mul_plain(a, p).data, "one-term product sum")
    with pytest.raises(he.HEError, match="levels"):
        g1.mac_plain([ga, gb], [gp, gp])
    half = g1.pt_from_numpy(p.data, p.scale * 2)
    with pytest.raises(he.HEError, match="scales"):
        g1.mac_plain([ga, ga], [gp, half])
    with pytest.raises(he.HEError, match="aliases"):
        g1.mac_plain([ga], [gp], out=ga)
    low = g1.pt_from_numpy(p.data[:3], p.scale)
    with pytest.raises(he.HEError, match="fewer limbs"):
        g1.mac_plain([ga], [low])
    with pytest.raises(he.HEError):
        g1.mul_i(ga, 0)
    with pytest.raises(he.HEError, match="aliases"):
        g1.mod_raise(ga, octx.pr.L, out=ga)
    with pytest.raises(he.HEError, match="range"):
        g1.mod_raise(ga, octx.pr.L + 1)
    x = g1.ct_from_numpy(a.data, a.scale)
    g1.mul_i(x, 1, out=x)
    H.assert_limbs_equal(x.numpy(), octx.mul_plain(a, BT.monomial_pt(octx, octx.n // 2, a.level)).data, "i in place")
    r1 = g1.mod_raise(ga, 1)
    H.assert_limbs_equal(r1.numpy(), a.data[:, :1], "raise to level 1")
