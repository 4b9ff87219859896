"""Dynamic key management: keys loaded on demand from host copies into a
device budget (LRU eviction), bit-exact against the oracle (needs MI355X)."""
import numpy as np
import pytest
import torch

import synth
from oracle import layers as LY
from tests import helpers as H
from tests.test_gpu_batch import make_batch, oracle_outputs

pytestmark = pytest.mark.gpu
NAME = "config1"


def fresh():
    return H.gpu_ctx(NAME)


def test_demand_loading_and_eviction():
    octx, _, _ = H.oracle_ctx(NAME)
    g = fresh()
    try:
        rots = [1, -3, 17, 200]
        for r in rots:
            g.key_host_register(r, H.oracle_key(NAME, r))
        g.key_cache_limit(2 * g.key_bytes())
        assert g.key_count() == 0
        _, ct = H.encrypt_slots(NAME, 80)
        gct = g.ct_from_numpy(ct.data, ct.scale)
        for rep in range(2):
            for r in rots:
                got = g.rotate(gct, r)
                H.assert_limbs_equal(got.numpy(), octx.rotate(ct, r, {r: H.oracle_key(NAME, r)}).data,
                                     "rotation %d under a 2-key budget (pass %d)" % (r, rep))
                assert g.key_cache_stats()["resident_bytes"] <= 2 * g.key_bytes()
        st = g.key_cache_stats()
        assert st["loads"] == 8 and st["evictions"] == 6, st
        # hoisted set of all four keys: the budget is exceeded by nothing evictable only transiently
        outs = g.rotate_hoisted(gct, rots)
        want = octx.rotate_hoisted(ct, rots, H.oracle_keys(NAME, rots))
        for o, w in zip(outs, want):
            H.assert_limbs_equal(o.numpy(), w.data, "hoisted set under a budget")
    finally:
        g.close()


def test_layer_under_budget():
    """Generic convolution (9 keys) with every key loaded on demand into a 3-key budget."""
    octx, sk, _ = H.oracle_ctx(NAME)
    slots = octx.n // 2
    g = fresh()
    try:
        X = synth.image(81, 2, 12, 12)
        K = synth.conv_weights(81, 3, 2, 3, 0.2)
        fm = LY.FMap(2, 12, 12)
        from paper_2510_03996_amd import he

        plan = g.conv2d_plan(he.he_fmap(*fm.key()), 3, 3, 1, 1)
        for r in plan.keys():
            g.key_host_register(r, H.oracle_key(NAME, r))
        g.key_cache_limit(3 * g.key_bytes())
        _, ct = H.encrypt_slots(NAME, 81, values=LY.pack(X, fm, slots))
        kern, masks = LY.conv_plaintexts(fm, K, 1, 1, slots)
        kp = [octx.encode(v, octx.pr.scale, ct.level) for v in kern]
        mp = [octx.encode(v, octx.pr.scale, ct.level) for v in masks]
        ev = LY.HEEval(octx, H.oracle_keys(NAME, plan.keys()))
        want, fo = LY.conv2d(ev, ct, fm, 3, 3, 1, 1, kp, mp, slots)
        got, _ = g.conv2d(g.ct_from_numpy(ct.data, ct.scale), he.he_fmap(*fm.key()), 3, 3, 1, 1,
                          [g.pt_from_numpy(p.data, p.scale) for p in kp], [g.pt_from_numpy(p.data, p.scale) for p in mp])
        H.assert_limbs_equal(got.numpy(), want.data, "convolution with keys loaded on demand")
        st = g.key_cache_stats()
        assert st["resident_bytes"] <= 3 * g.key_bytes() and st["evictions"] > 0, st
    finally:
        g.close()


def test_batch_holds_its_keys():
    from paper_2510_03996_amd import he

    octx, sets, outs, cts, pool, pti = make_batch(NAME, 3, 4, 2, 3, 1, 2, seed=82)
    g = fresh()
    try:
        keys = sorted({r for s in sets for r in s})
        for r in keys:
            g.key_host_register(r, H.oracle_key(NAME, r))
        g.key_cache_limit(g.key_bytes())  # smaller than the batch's key set: the budget is soft for held keys
        level = cts[0].level
        inp = he.to_device(np.stack([c.data for c in cts]))
        pt = he.to_device(np.stack([p.data for p in pool]))
        out = torch.zeros((sum(outs), 2, level - 1, g.n), dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        b = he.Batch(g, inp, level, cts[0].scale, sets, outs, pt, pool[0].scale, pti, out, he.BATCH_GRAPH)
        assert g.key_count() == len(keys)
        with pytest.raises(he.HEError) as e:
            g.key_evict(keys[0])
        assert e.value.name == "HE_EINVAL"
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            b.run(s)
            s.synchronize()
        want = oracle_outputs(NAME, sets, outs, cts, pool, pti)
        got = out.cpu().numpy().view(np.uint64)
        for i, w in enumerate(want):
            H.assert_limbs_equal(got[i], w.data, "batched output %d with held keys" % i)
        b.close()
        g.key_evict(keys[0])  # no longer held
    finally:
        g.close()


def test_prefetch_on_another_stream():
    octx, _, _ = H.oracle_ctx(NAME)
    g = fresh()
    try:
        g.key_host_register(5, H.oracle_key(NAME, 5))
        a, b = torch.cuda.Stream(), torch.cuda.Stream()
        _, ct = H.encrypt_slots(NAME, 83)
        gct = g.ct_from_numpy(ct.data, ct.scale)
        out = g.new_ct(ct.level)
        torch.cuda.synchronize()
        g.key_prefetch([5], stream=a)  # loaded on stream a ...
        g.rotate(gct, 5, out=out, stream=b)  # ... and used at once on stream b, which waits for the load
        b.synchronize()
        H.assert_limbs_equal(out.numpy(), octx.rotate(ct, 5, {5: H.oracle_key(NAME, 5)}).data, "prefetched key")
        assert g.key_cache_stats()["loads"] == 1
    finally:
        torch.cuda.synchronize()
        g.close()


def _keep_busy(stream):
    """Enqueue several milliseconds of bounded work on `stream`."""
    with torch.cuda.stream(stream):
        if hasattr(torch.cuda, "_sleep"):
            torch.cuda._sleep(20_000_000)
        else:
            x = torch.ones(64 << 20, device="cuda")
            for _ in range(20):
                x.mul_(1.0)


def test_eviction_waits_for_every_stream():
    """With a one-key budget, a key still read by work queued on stream a must
    not be evicted (its buffer reloaded) because stream b's use of it is done."""
    octx, _, _ = H.oracle_ctx(NAME)
    g = fresh()
    try:
        k1, k2 = 3, -9
        for r in (k1, k2):
            g.key_host_register(r, H.oracle_key(NAME, r))
        g.key_cache_limit(g.key_bytes())
        _, ct = H.encrypt_slots(NAME, 84)
        gct = g.ct_from_numpy(ct.data, ct.scale)
        want1 = octx.rotate(ct, k1, {k1: H.oracle_key(NAME, k1)}).data
        want2 = octx.rotate(ct, k2, {k2: H.oracle_key(NAME, k2)}).data
        a, b = torch.cuda.Stream(), torch.cuda.Stream()
        outs_a = [g.new_ct(ct.level) for _ in range(8)]
        out_b1, out_b2 = g.new_ct(ct.level), g.new_ct(ct.level)
        g.lane_reserve(a, 1)  # no allocation once the busy work is queued
        g.lane_reserve(b, 1)
        g.key_prefetch([k1])
        torch.cuda.synchronize()
        _keep_busy(a)
        for o in outs_a:  # queued behind the busy work: they read k1 later
            g.rotate(gct, k1, out=o, stream=a)
        g.rotate(gct, k1, out=out_b1, stream=b)  # runs at once
        b.synchronize()
        g.rotate(gct, k2, out=out_b2, stream=b)  # evicts k1: must wait for stream a's reads
        torch.cuda.synchronize()
        for i, o in enumerate(outs_a):
            H.assert_limbs_equal(o.numpy(), want1, "rotation %d queued on the other stream" % i)
        H.assert_limbs_equal(out_b1.numpy(), want1, "rotation on stream b")
        H.assert_limbs_equal(out_b2.numpy(), want2, "rotation with the reloaded buffer")
        assert g.key_cache_stats()["evictions"] >= 1
    finally:
        torch.cuda.synchronize()
        g.close()


def test_convolution_streams_under_budget():
    """Special convolution at N=2^16 (four replicated channels of 64x64, 20 key
    switches) on four layer streams with every key loaded on demand into a
    two-key budget: the hoisted taps and the channel sums on different streams
    evict and reload keys that other streams have read; bit-exact."""
    from paper_2510_03996_amd import he

    name = "config2"
    octx, _, _ = H.oracle_ctx(name)
    slots = octx.n // 2
    g = H.gpu_ctx(name)
    try:
        X = synth.image(23, 4, 64, 64)
        K = synth.conv_weights(23, 4, 4, 3, (2.0 / 36) ** 0.5)
        fm = LY.FMap(4, 64, 64, reps=2)
        hfm = he.he_fmap(*fm.key())
        plan = g.conv2d_plan(hfm, 4, 3, 1, 1)
        for r in plan.keys():
            g.key_host_register(r, H.oracle_key(name, r))
        g.key_cache_limit(2 * g.key_bytes())
        g.layer_streams(4)
        _, ct = H.encrypt_slots(name, 85, values=LY.pack(X, fm, slots))
        kern, masks = LY.conv_plaintexts(fm, K, 1, 1, slots)
        kp = [octx.encode(v, octx.pr.scale, ct.level) for v in kern]
        mp = [octx.encode(v, octx.pr.scale, ct.level) for v in masks]
        ev = LY.HEEval(octx, H.oracle_keys(name, plan.keys()))
        want, _ = LY.conv2d(ev, ct, fm, 4, 3, 1, 1, kp, mp, slots)
        got, _ = g.conv2d(g.ct_from_numpy(ct.data, ct.scale), hfm, 4, 3, 1, 1,
                          [g.pt_from_numpy(p.data, p.scale) for p in kp], [g.pt_from_numpy(p.data, p.scale) for p in mp])
        torch.cuda.synchronize()
        H.assert_limbs_equal(got.numpy(), want.data, "convolution on four streams with keys loaded on demand")
        st = g.key_cache_stats()
        assert st["evictions"] > 0 and st["resident_bytes"] <= 2 * g.key_bytes(), st
    finally:
        torch.cuda.synchronize()
        g.close()


def test_key_cache_errors():
    from paper_2510_03996_amd import he

    g = fresh()
    try:
        with pytest.raises(he.HEError) as e:
            g.key_cache_limit(g.key_bytes() - 8)
        assert e.value.name == "HE_EINVAL"
        with pytest.raises(he.HEError) as e:
            g.key_prefetch([99])
        assert e.value.name == "HE_ENOKEY"
        with pytest.raises(he.HEError) as e:
            g.key_host_register(7, np.zeros(16, dtype=np.uint64))
        assert e.value.name == "HE_EINVAL"
    finally:
        g.close()
