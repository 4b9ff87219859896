"""Batched hoisted-rotation MAC: batched schedule == per-op path == oracle, bit for bit (needs MI355X)."""
import numpy as np
import pytest
import torch

import synth
from oracle import ckks
from tests import helpers as H

pytestmark = pytest.mark.gpu


def make_batch(name, B, pool_n, n_lo, n_hi, m_lo, m_hi, seed, level=None, pool_offsets=None):
    octx, _, _ = H.oracle_ctx(name)
    pr = octx.pr
    level = level or pr.L
    pool_offsets = pool_offsets or [1, -1, 2, -2, 3, 5, 7, 16, -16, 32]
    sets, outs = synth.rotation_sets(seed, B, pool_offsets, n_lo, n_hi, m_lo, m_hi)
    cts = [H.encrypt_slots(name, seed * 100 + i, level=level, enc_id=i)[1] for i in range(B)]
    pool = [octx.encode(synth.uniform_slots(seed * 1000 + p, pr.n // 2, stream=9), pr.scale, level)
            for p in range(pool_n)]
    # pt index for (i, o, t): pool[(i + 7 o + 13 t) mod pool_n]
    pti = [[(i + 7 * o + 13 * t) % pool_n for o in range(outs[i]) for t in range(len(sets[i]))] for i in range(B)]
    return octx, sets, outs, cts, pool, pti


def run_gpu(g, name, sets, outs, cts, pool, pti, flags):
    from paper_2510_03996_amd import he

    level = cts[0].level
    keys = sorted({r for s in sets for r in s})
    for r in keys:
        g.key_upload(r, H.oracle_key(name, r))
    inp = he.to_device(np.stack([c.data for c in cts]))
    pt = he.to_device(np.stack([p.data for p in pool]))
    total = sum(outs)
    out_b = torch.zeros((total, 2, level - 1, g.n), dtype=torch.int64, device="cuda")
    out_p = torch.zeros_like(out_b)
    b = he.Batch(g, inp, level, cts[0].scale, sets, outs, pt, pool[0].scale, pti, out_b, flags)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.run(s)
        b.run(s)  # graph replay (if enabled) must give the same result
        s.synchronize()
        got_b = out_b.cpu().numpy().view(np.uint64).copy()
        b2 = he.Batch(g, inp, level, cts[0].scale, sets, outs, pt, pool[0].scale, pti, out_p, 0)
        b2.run_plain(s)
        s.synchronize()
    got_p = out_p.cpu().numpy().view(np.uint64)
    info = b.info()
    b.close()
    b2.close()
    return got_b, got_p, info


def oracle_outputs(name, sets, outs, cts, pool, pti):
    octx, _, _ = H.oracle_ctx(name)
    res = []
    for i, ct in enumerate(cts):
        keys = H.oracle_keys(name, sets[i])
        rot = octx.rotate_hoisted(ct, sets[i], keys)
        n = len(sets[i])
        for o in range(outs[i]):
            acc = None
            for t in range(n):
                m = octx.mul_plain(rot[t], pool[pti[i][o * n + t]])
                acc = m if acc is None else octx.add(acc, m)
            res.append(octx.rescale(acc))
    return res


@pytest.mark.parametrize("name,flags", [("config1", 0), ("config1", 1), ("config1", 2), ("config2", 5)])
def test_batch_matches_plain_and_oracle(name, flags):
    B = 3 if name == "config2" else 5
    octx, sets, outs, cts, pool, pti = make_batch(name, B, 6, 2, 4, 1, 3, seed=31)
    g = H.gpu_ctx(name)
    got_b, got_p, info = run_gpu(g, name, sets, outs, cts, pool, pti, flags)
    assert info["rotations"] == sum(len(s) for s in sets) and info["outputs"] == sum(outs)
    H.assert_limbs_equal(got_b, got_p, "batched vs plain")
    want = oracle_outputs(name, sets, outs, cts, pool, pti)
    for k, w in enumerate(want):
        H.assert_limbs_equal(got_b[k], w.data, "batched vs oracle output %d" % k)
    assert info["out_scale"] == want[0].scale
    g.close()


@pytest.mark.parametrize("variant", range(5))
def test_batch_every_mac_variant(variant):
    """Every register grouping of the batched MAC (outputs per group x
    polynomials per workgroup) equals the per-op path and the oracle, on
    items with up to 40 outputs (several groups for every variant)."""
    from paper_2510_03996_amd import he

    name = "config1"
    octx, sets, outs, cts, pool, pti = make_batch(name, 4, 6, 2, 4, 1, 3, seed=53)
    outs[0], outs[2] = 40, 17
    pti = [[(i + 7 * o + 13 * t) % 6 for o in range(outs[i]) for t in range(len(sets[i]))] for i in range(4)]
    g = H.gpu_ctx(name)
    got_b, got_p, info = run_gpu(g, name, sets, outs, cts, pool, pti, he.batch_mac_select(variant) | 1)
    H.assert_limbs_equal(got_b, got_p, "batched (MAC variant %d) vs plain" % variant)
    want = oracle_outputs(name, sets, outs, cts, pool, pti)
    for k in (0, 39, 40, 41, len(want) - 1):
        H.assert_limbs_equal(got_b[k], want[k].data, "batched vs oracle output %d" % k)
    g.close()


def test_batch_larger_config2_batched_equals_plain():
    """16 ciphertexts at N=2^16, L=24, 9-15 rotations from a 7x7-window pool, 1-8 outputs."""
    name = "config2"
    pool_offsets = [dy * 32 + dx for dy in range(-3, 4) for dx in range(-3, 4) if (dy, dx) != (0, 0)]
    octx, sets, outs, cts, pool, pti = make_batch(name, 16, 8, 9, 15, 1, 8, seed=37, pool_offsets=pool_offsets)
    g = H.gpu_ctx(name)
    got_b, got_p, info = run_gpu(g, name, sets, outs, cts, pool, pti, 1)
    H.assert_limbs_equal(got_b, got_p, "batched vs plain")
    g.close()


def test_batch_mac_extreme_residues():
    """The batched MAC's centred FP64 products (primes below 2^50) and its
    integer path (q_0) against the per-op path's Barrett products, with
    plaintext residues at the edges of their range (0, 1, q - 1, q/2, q/2 + 1)
    and 9-17 terms per output so that the sums pass through several
    re-centrings."""
    name = "config2"
    offsets = [1, -1, 2, -2, 3, -3, 4, -4, 5, -5, 7, -7, 16, -16, 32, -32, 64]
    octx, sets, outs, cts, pool, pti = make_batch(name, 3, 4, 9, 17, 1, 3, seed=41, pool_offsets=offsets)
    q = octx.pr.q
    for p, pt in enumerate(pool):
        d = pt.data
        k = np.arange(d.shape[1])
        for i in range(d.shape[0]):
            qi = np.uint64(q[i])
            edge = np.array([0, 1, q[i] - 1, q[i] // 2, q[i] // 2 + 1], dtype=np.uint64)
            sel = (k + p + i) % 7
            d[i] = np.where(sel < 5, edge[np.minimum(sel, 4)], d[i] % qi)
    from paper_2510_03996_amd import he

    g = H.gpu_ctx(name)
    for v in (0, 4):  # both polynomials per workgroup, and one
        got_b, got_p, info = run_gpu(g, name, sets, outs, cts, pool, pti, he.batch_mac_select(v))
        H.assert_limbs_equal(got_b, got_p, "batched (MAC variant %d) vs plain, extreme plaintext residues" % v)
    g.close()


def test_batch_config3_shape_matches_oracle():
    """The batched workload's shape at N=2^16, L=24 against the oracle: 8
    ciphertexts with hoisted sets from the 49-key pool (the 48 non-zero
    offsets of a 7x7 window on a 32-wide map, plus 1024), one item rotated by
    all 49 keys, one with 32 outputs, the others 9-12 rotations and 1-4
    outputs; every output limb compared with the oracle's
    rotate_hoisted + mul_plain + add + rescale."""
    name = "config2"
    pool_offsets = [dy * 32 + dx for dy in range(-3, 4) for dx in range(-3, 4) if (dy, dx) != (0, 0)] + [1024]
    octx, _, _ = H.oracle_ctx(name)
    pr = octx.pr
    B, pool_n, seed = 8, 16, 43
    sets, outs = synth.rotation_sets(seed, B, pool_offsets, 9, 12, 1, 4)
    sets[0] = [int(x) for x in synth.rng(seed, 11).permutation(np.asarray(pool_offsets))]  # n = 49
    outs[1] = 32  # m = 32
    cts = [H.encrypt_slots(name, seed * 100 + i, level=pr.L, enc_id=i)[1] for i in range(B)]
    pool = [octx.encode(synth.uniform_slots(seed * 1000 + p, pr.n // 2, stream=9), pr.scale, pr.L)
            for p in range(pool_n)]
    pti = [[(i + 7 * o + 13 * t) % pool_n for o in range(outs[i]) for t in range(len(sets[i]))] for i in range(B)]
    print("config-3 shape: n =", [len(s) for s in sets], "m =", outs, flush=True)
    g = H.gpu_ctx(name)
    got_b, got_p, info = run_gpu(g, name, sets, outs, cts, pool, pti, 5)
    assert info["keys"] == 49 and info["rotations"] == sum(len(s) for s in sets)
    H.assert_limbs_equal(got_b, got_p, "batched vs plain")
    want = oracle_outputs(name, sets, outs, cts, pool, pti)
    assert len(want) == got_b.shape[0]
    for k, w in enumerate(want):
        H.assert_limbs_equal(got_b[k], w.data, "batched vs oracle output %d" % k)
    assert info["out_scale"] == want[0].scale
    g.close()
