"""Continuous-batching serving: every result is the same alone and in the mix (needs MI355X)."""
import numpy as np
import pytest
import torch

import synth
from oracle import ckks
from oracle import layers as LY
from tests import helpers as H

pytestmark = pytest.mark.gpu


def lenet_real(name="config1"):
    """LeNet-5-shaped model with oracle keys and oracle-encoded weights."""
    from paper_2510_03996_amd import he, models, serve

    octx, sk, pk = H.oracle_ctx(name)
    slots = octx.n // 2
    g = H.gpu_ctx(name)
    fm0, pc, pp, keys = models.lenet_plan(g)
    for r in keys:
        g.key_upload(r, H.oracle_key(name, r))
    g.key_upload(he.KEY_RELIN, H.oracle_key(name, "relin"))
    K = synth.conv_weights(40, 6, 1, 5, 0.1)
    fm = LY.FMap(1, 28, 28)
    f1 = LY.conv_out_map(fm, 6, 5, 1, 0, slots)
    # the library's own recipes (equal to the oracle's, tests/test_host_plaintexts.py);
    # the client-side encoding is the oracle's
    kern, pool = models.lenet_vectors(K)
    assert len(kern) == pc.n_kernel_pts and len(pool) == pp.n_mask_pts
    L = octx.pr.L
    kp = [g.pt_from_numpy(octx.encode(v, octx.pr.scale, L).data, octx.pr.scale) for v in kern]
    mp = [g.pt_from_numpy(octx.encode(v, octx.pr.scale, L).data, octx.pr.scale) for v in pool]
    chain = models.lenet_chain(g, kp, mp, octx.pr.scale)
    model = serve.Model("lenet", g, chain.stages, 16, g.lane_bytes(16))
    return g, model, K, f1


def test_serve_lenet_alone_vs_mix_decrypts():
    from paper_2510_03996_amd import serve

    name = "config1"
    octx, sk, _ = H.oracle_ctx(name)
    g, model, K, f1 = lenet_real(name)
    fm = LY.FMap(1, 28, 28)
    imgs = [synth.image(50 + i, 1, 28, 28) for i in range(6)]
    cts = [H.encrypt_slots(name, 50 + i, enc_id=i, values=LY.pack(X, fm, octx.n // 2))[1] for i, X in enumerate(imgs)]
    srv = serve.Server({"lenet": model}, slots=3)

    def reqs():
        return [serve.Request(i, "lenet", 0.0, g.ct_from_numpy(c.data, c.scale)) for i, c in enumerate(cts)]

    alone = sorted(srv.serve(reqs(), "sequential"), key=lambda r: r.id)
    mix = sorted(srv.serve(reqs(), "continuous"), key=lambda r: r.id)
    assert srv.max_active == 3
    f2 = LY.FMap(6, 12, 12)
    for a, m, X in zip(alone, mix, imgs):
        H.assert_limbs_equal(m.output.numpy(), a.output.numpy(), "request %d alone vs mix" % a.id)
        dec = LY.unpack(octx.decrypt(sk, ckks.Ciphertext(m.output.numpy(), m.output.scale)), f2)
        ref = LY.avgpool_ref(LY.relu4_ref(LY.conv2d_ref(X, K, 1, 0)), 2, 2)
        assert np.max(np.abs(dec - ref)) < 1e-2
    srv.close()
    g.close()


def test_serve_mixed_rings_synthetic_alone_vs_mix():
    """LeNet-shaped (N=2^14) and ResNet-shaped (N=2^16) requests in one mix,
    synthetic keys and weights; also a budget that forces queueing."""
    import bench
    from paper_2510_03996_amd import serve

    models, make_input = bench.synthetic_serving_models(seed=5)
    srv = serve.Server(models, slots=3)
    kinds = ["lenet", "resnet", "lenet", "lenet", "resnet", "lenet"]
    inputs = [make_input(k, 100 + i) for i, k in enumerate(kinds)]

    def reqs():
        return [serve.Request(i, k, 0.002 * i, inputs[i]) for i, k in enumerate(kinds)]

    alone = sorted(srv.serve(reqs(), "sequential"), key=lambda r: r.id)
    mix = sorted(srv.serve(reqs(), "continuous"), key=lambda r: r.id)
    assert srv.max_active >= 2
    for a, m in zip(alone, mix):
        H.assert_limbs_equal(m.output.numpy(), a.output.numpy(), "request %d (%s)" % (a.id, a.kind))
    srv.close()
    # a budget that fits one request at a time: still correct, never two in flight
    tight = serve.Server(models, slots=3, budget_bytes=min(m.footprint for m in models.values()))
    queued = sorted(tight.serve(reqs(), "continuous"), key=lambda r: r.id)
    assert tight.max_active == 1
    for a, q in zip(alone, queued):
        H.assert_limbs_equal(q.output.numpy(), a.output.numpy(), "budgeted request %d" % a.id)
    tight.close()
    for m in models.values():
        m.ctx.close()
