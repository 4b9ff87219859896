"""GPU vs oracle parity for the CKKS ops, bit-exact on every limb (needs MI355X)."""
import numpy as np
import pytest

from oracle import _lib as OC
from oracle import ckks
from tests import helpers as H

pytestmark = pytest.mark.gpu

CONFIGS = ["config0", "config1", "config2"]


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


@pytest.mark.parametrize("name", CONFIGS)
def test_moduli_match_oracle(gctx, name):
    octx, _, _ = H.oracle_ctx(name)
    assert gctx(name).moduli == octx.pr.moduli


@pytest.mark.parametrize("name", CONFIGS)
def test_ntt_forward_inverse(gctx, name):
    import synth
    from paper_2510_03996_amd import he

    g = gctx(name)
    octx, _, _ = H.oracle_ctx(name)
    pr = octx.pr
    a = synth.residues(1, pr.moduli, pr.n)
    t = he.to_device(a)
    g.ntt(t, 0, inverse=False)
    want = OC.ntt(a, pr.moduli, pr.psi)
    H.assert_limbs_equal(t.cpu().numpy().view(np.uint64), want, "forward NTT")
    g.ntt(t, 0, inverse=True)
    H.assert_limbs_equal(t.cpu().numpy().view(np.uint64), a, "NTT round trip")
    # a sub-range of limbs, special primes included
    b = a[pr.L - 1:]
    tb = he.to_device(b)
    g.ntt(tb, pr.L - 1, inverse=True)
    H.assert_limbs_equal(tb.cpu().numpy().view(np.uint64), OC.ntt(b, pr.moduli[pr.L - 1:], pr.psi[pr.L - 1:], True),
                         "inverse NTT on q_top..p_K")


@pytest.mark.parametrize("name", CONFIGS)
def test_every_ntt_variant(gctx, name):
    """Each (tile, residues per thread) kernel shape, pinned in turn for every
    batch-size bucket: forward NTT, round trip and a full key-switch rotation."""
    import synth
    from paper_2510_03996_amd import he

    g = gctx(name)
    octx, _, _ = H.oracle_ctx(name)
    pr = octx.pr
    tuned = g.ntt_variants()
    a = synth.residues(11, pr.moduli, pr.n)
    want = OC.ntt(a, pr.moduli, pr.psi)
    g.key_upload(5, H.oracle_key(name, 5))
    _, ct = H.encrypt_slots(name, 12)
    want_rot = octx.rotate(ct, 5, {5: H.oracle_key(name, 5)})
    try:
        for v in range(he.NTT_VARIANTS):
            g.ntt_select([v] * 4)
            t = he.to_device(a)
            g.ntt(t, 0, inverse=False)
            H.assert_limbs_equal(t.cpu().numpy().view(np.uint64), want, "forward NTT, variant %d" % v)
            g.ntt(t, 0, inverse=True)
            H.assert_limbs_equal(t.cpu().numpy().view(np.uint64), a, "round trip, variant %d" % v)
            got = g.rotate(g.ct_from_numpy(ct.data, ct.scale), 5)
            H.assert_limbs_equal(got.numpy(), want_rot.data, "rotation, variant %d" % v)
    finally:
        g.ntt_select(tuned)
        g.key_evict(5)  # the module's contexts are shared: leave the key set as found
    with pytest.raises(he.HEError):
        g.ntt_select([0, 0, 0, he.NTT_VARIANTS])
    assert g.ntt_variants() == tuned


@pytest.mark.parametrize("name", CONFIGS)
def test_pointwise_and_rescale(gctx, name):
    g = gctx(name)
    octx, _, _ = H.oracle_ctx(name)
    pr = octx.pr
    _, a = H.encrypt_slots(name, 1, enc_id=0)
    _, b = H.encrypt_slots(name, 2, enc_id=1)
    _, pt = H.encode_slots(name, 3, pr.L)
    ga, gb = g.ct_from_numpy(a.data, a.scale), g.ct_from_numpy(b.data, b.scale)
    gpt = g.pt_from_numpy(pt.data, pt.scale)
    H.assert_limbs_equal(g.add(ga, gb).numpy(), octx.add(a, b).data, "add")
    H.assert_limbs_equal(g.sub(ga, gb).numpy(), octx.sub(a, b).data, "sub")
    want_ap = octx.add_plain(a, ckks.Plaintext(pt.data, a.scale))
    H.assert_limbs_equal(g.add_plain(ga, g.pt_from_numpy(pt.data, a.scale)).numpy(), want_ap.data, "add_plain")
    m = g.mul_plain(ga, gpt)
    om = octx.mul_plain(a, pt)
    H.assert_limbs_equal(m.numpy(), om.data, "mul_plain")
    assert m.scale == om.scale
    acc = g.mul_plain(ga, gpt)
    g.mul_plain(gb, gpt, out=acc, accumulate=True)
    H.assert_limbs_equal(acc.numpy(), octx.add(om, octx.mul_plain(b, pt)).data, "mul_plain accumulate")
    r = g.rescale(m)
    orr = octx.rescale(om)
    H.assert_limbs_equal(r.numpy(), orr.data, "rescale")
    assert r.level == orr.level and r.scale == orr.scale
    # in-place rescale
    g.rescale(m, out=m)
    H.assert_limbs_equal(m.numpy(), orr.data, "rescale in place")
    d = g.drop_level(ga, max(1, pr.L - 2))
    H.assert_limbs_equal(d.numpy(), octx.drop_level(a, max(1, pr.L - 2)).data, "drop_level")


@pytest.mark.parametrize("name,n,level", [("config0", 3, None), ("config1", 19, 5), ("config2", 9, None)])
def test_mac_plain(gctx, name, n, level):
    """he_mac_plain (one pass; 19 terms exceed one launch's 16) against the
    oracle's sum of products, fresh and accumulating."""
    g = gctx(name)
    octx, _, _ = H.oracle_ctx(name)
    pr = octx.pr
    lv = level or pr.L
    cts = [H.encrypt_slots(name, 40 + t, level=lv, enc_id=t)[1] for t in range(n)]
    pts = [H.encode_slots(name, 60 + t, pr.L)[1] for t in range(n)]
    want = octx.mul_plain(cts[0], pts[0])
    for c, p in zip(cts[1:], pts[1:]):
        want = octx.add(want, octx.mul_plain(c, p))
    gcts = [g.ct_from_numpy(c.data, c.scale) for c in cts]
    gpts = [g.pt_from_numpy(p.data, p.scale) for p in pts]
    got = g.mac_plain(gcts, gpts)
    H.assert_limbs_equal(got.numpy(), want.data, "mac_plain")
    assert got.level == want.level and got.scale == want.scale
    g.mac_plain(gcts[:2], gpts[:2], out=got, accumulate=True)
    want2 = octx.add(want, octx.add(octx.mul_plain(cts[0], pts[0]), octx.mul_plain(cts[1], pts[1])))
    H.assert_limbs_equal(got.numpy(), want2.data, "mac_plain accumulate")


ROTS = {"config0": [1, -1, 7, -512], "config1": [1, -28, 576, -3], "config2": [1, -1, 32, -1024]}


@pytest.mark.parametrize("name", CONFIGS)
def test_rotate_single(gctx, name):
    g = gctx(name)
    octx, _, _ = H.oracle_ctx(name)
    r = ROTS[name][0]
    key = H.oracle_key(name, r)
    g.key_upload(r, key)
    _, a = H.encrypt_slots(name, 11)
    got = g.rotate(g.ct_from_numpy(a.data, a.scale), r)
    want = octx.rotate(a, r, {r: key})
    H.assert_limbs_equal(got.numpy(), want.data, "rotate %d" % r)
    assert got.scale == want.scale and got.level == want.level


@pytest.mark.parametrize("name", CONFIGS)
def test_rotate_single_every_key(gctx, name):
    """One key switch per call takes the path with the inner product fused
    into ModUp's last NTT pass: every rotation of the set (its own Galois
    element, so its own tile mapping), and a hoisted call with one non-zero
    rotation."""
    g = gctx(name)
    octx, _, _ = H.oracle_ctx(name)
    keys = H.oracle_keys(name, ROTS[name])
    for r, k in keys.items():
        g.key_upload(r, k)
    _, a = H.encrypt_slots(name, 14)
    ga = g.ct_from_numpy(a.data, a.scale)
    for r in ROTS[name]:
        H.assert_limbs_equal(g.rotate(ga, r).numpy(), octx.rotate(a, r, {r: keys[r]}).data, "rotate %d" % r)
    r = ROTS[name][-1]
    got = g.rotate_hoisted(ga, [0, r])
    want = octx.rotate_hoisted(a, [0, r], {r: keys[r]})
    for x, y in zip(got, want):
        H.assert_limbs_equal(x.numpy(), y.data, "hoisted [0, %d]" % r)


@pytest.mark.parametrize("name", CONFIGS)
def test_rotate_hoisted(gctx, name):
    g = gctx(name)
    octx, _, _ = H.oracle_ctx(name)
    rs = ROTS[name] + [0]
    keys = H.oracle_keys(name, ROTS[name])
    for r, k in keys.items():
        g.key_upload(r, k)
    _, a = H.encrypt_slots(name, 12)
    ga = g.ct_from_numpy(a.data, a.scale)
    want = octx.rotate_hoisted(a, rs, keys)
    # the key switches of the set on 1, 2, 3 and 8 streams (caller + helpers)
    for n in (1, 2, 3, 8):
        g.layer_streams(n)
        got = g.rotate_hoisted(ga, rs)
        for r, x, y in zip(rs, got, want):
            H.assert_limbs_equal(x.numpy(), y.data, "hoisted rotation %d on %d stream(s)" % (r, n))
    g.layer_streams(2)


@pytest.mark.parametrize("level", [24, 13])
def test_rotate_hoisted_rounds(gctx, level):
    """A hoisted set of 13 key switches (the 3x3 window's 8 offsets on a
    32-wide map, four more, and the identity) at N=2^16: two rounds of the
    batched set path (8 + 5), spread over 1, 2 and 4 streams; at level 13 the
    last digit is partial (8 + 5 limbs).  Every output equals the oracle's."""
    name = "config2"
    g = gctx(name)
    octx, _, _ = H.oracle_ctx(name)
    rs = [dy * 32 + dx for dy in (-1, 0, 1) for dx in (-1, 0, 1) if (dy, dx) != (0, 0)] + [2, -64, 1024, 4095, 0]
    ks = [r for r in rs if r != 0]
    keys = H.oracle_keys(name, ks)
    for r, k in keys.items():
        g.key_upload(r, k)
    _, a = H.encrypt_slots(name, 15, level=level)
    ga = g.ct_from_numpy(a.data, a.scale)
    want = octx.rotate_hoisted(a, rs, keys)
    for n in (1, 2, 4):
        g.layer_streams(n)
        got = g.rotate_hoisted(ga, rs)
        for r, x, y in zip(rs, got, want):
            H.assert_limbs_equal(x.numpy(), y.data, "hoisted rotation %d at level %d on %d stream(s)" % (r, level, n))
            assert x.level == level
    g.layer_streams(2)


def test_helper_streams_released_with_the_lane(gctx):
    """A hoisted set on a fresh stream (its key switches over the stream and a
    helper), the stream's lane released (helpers destroyed), the same set
    again on that stream (helpers recreated): both equal the oracle."""
    import torch

    name = "config2"
    g = gctx(name)
    octx, _, _ = H.oracle_ctx(name)
    rs = ROTS[name]
    keys = H.oracle_keys(name, rs)
    for r, k in keys.items():
        g.key_upload(r, k)
    _, a = H.encrypt_slots(name, 14)
    ga = g.ct_from_numpy(a.data, a.scale)
    want = octx.rotate_hoisted(a, rs, keys)
    st = torch.cuda.Stream()
    g.layer_streams(2)
    for rep in range(2):
        got = g.rotate_hoisted(ga, rs, stream=st)
        st.synchronize()
        for r, x, y in zip(rs, got, want):
            H.assert_limbs_equal(x.numpy(), y.data, "hoisted rotation %d, pass %d" % (r, rep))
        g.lane_release(st)


@pytest.mark.parametrize("name,level", [("config2", 13), ("config2", 8), ("config1", 5), ("config1", 2), ("config0", 2)])
def test_rotate_lower_levels(gctx, name, level):
    """Partial last digit and restricted keys at lower levels."""
    g = gctx(name)
    octx, _, _ = H.oracle_ctx(name)
    r = ROTS[name][1]
    key = H.oracle_key(name, r)
    g.key_upload(r, key)
    _, a = H.encrypt_slots(name, 13, level=level)
    got = g.rotate(g.ct_from_numpy(a.data, a.scale, cap=octx.pr.L), r)
    H.assert_limbs_equal(got.numpy(), octx.rotate(a, r, {r: key}).data, "rotate at level %d" % level)


@pytest.mark.parametrize("name", CONFIGS)
def test_mul_relin(gctx, name):
    g = gctx(name)
    octx, _, _ = H.oracle_ctx(name)
    rk = H.oracle_key(name, "relin")
    from paper_2510_03996_amd import he

    g.key_upload(he.KEY_RELIN, rk)
    _, a = H.encrypt_slots(name, 21, enc_id=0)
    _, b = H.encrypt_slots(name, 22, enc_id=1)
    got = g.mul_relin(g.ct_from_numpy(a.data, a.scale), g.ct_from_numpy(b.data, b.scale))
    want = octx.mul_relin(a, b, rk)
    H.assert_limbs_equal(got.numpy(), want.data, "mul_relin")
    assert got.scale == want.scale


def test_decrypted_rotation_semantics(gctx):
    """Decrypting the GPU's rotation gives roll(v, -r) (paper's Rot direction)."""
    name = "config1"
    g = gctx(name)
    octx, sk, _ = H.oracle_ctx(name)
    r = ROTS[name][1]
    g.key_upload(r, H.oracle_key(name, r))
    v, a = H.encrypt_slots(name, 31)
    got = g.rotate(g.ct_from_numpy(a.data, a.scale), r)
    dec = octx.decrypt(sk, ckks.Ciphertext(got.numpy(), got.scale))
    assert np.max(np.abs(dec - np.roll(v, -r))) < 1e-5


def test_error_codes(gctx):
    from paper_2510_03996_amd import he

    name = "config0"
    g = gctx(name)
    _, a = H.encrypt_slots(name, 41)
    ga = g.ct_from_numpy(a.data, a.scale)
    with pytest.raises(he.HEError) as e:
        g.rotate(ga, 3)  # key for 3 never uploaded
    assert e.value.name == "HE_ENOKEY"
    low = g.drop_level(ga, 2)
    with pytest.raises(he.HEError) as e:
        g.add(ga, low)
    assert e.value.name == "HE_ELEVEL"
    ga2 = g.ct_from_numpy(a.data, a.scale * 2)
    with pytest.raises(he.HEError) as e:
        g.add(ga, ga2)
    assert e.value.name == "HE_ESCALE"
    one = g.drop_level(ga, 1)
    with pytest.raises(he.HEError) as e:
        g.rescale(one)
    assert e.value.name == "HE_ELEVEL"
    with pytest.raises(he.HEError) as e:
        g.rotate_hoisted(ga, [1], outs=[ga])
    assert e.value.name == "HE_EINVAL"


# six one-limb digits: more digits than the fused inner-product kernel takes,
# so single and hoisted key switches use the separate ModUp / inner product
ckks.CONFIGS.setdefault("dnum6", dict(log_n=12, q_bits=[50, 45, 45, 45, 45, 45], p_bits=[55], alpha=1,
                                      log_scale=40))


def test_key_switch_many_digits():
    name = "dnum6"
    g = H.gpu_ctx(name)
    octx, _, _ = H.oracle_ctx(name)
    from paper_2510_03996_amd import he

    rs = [3, -100]
    keys = H.oracle_keys(name, rs)
    for r, k in keys.items():
        g.key_upload(r, k)
    rk = H.oracle_key(name, "relin")
    g.key_upload(he.KEY_RELIN, rk)
    _, a = H.encrypt_slots(name, 41)
    _, b = H.encrypt_slots(name, 42, enc_id=1)
    ga = g.ct_from_numpy(a.data, a.scale)
    H.assert_limbs_equal(g.rotate(ga, rs[0]).numpy(), octx.rotate(a, rs[0], keys).data, "rotate, 6 digits")
    got = g.rotate_hoisted(ga, rs)
    for x, y in zip(got, octx.rotate_hoisted(a, rs, keys)):
        H.assert_limbs_equal(x.numpy(), y.data, "hoisted, 6 digits")
    m = g.mul_relin(ga, g.ct_from_numpy(b.data, b.scale))
    H.assert_limbs_equal(m.numpy(), octx.mul_relin(a, b, rk).data, "mul_relin, 6 digits")
    g.close()
