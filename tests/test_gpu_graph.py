"""Graph capture of library calls (needs MI355X): a captured bootstrap (its
hoisted sets, key switches, products, rescales and the Chebyshev evaluation,
with helper streams forked and joined inside the capture) and a captured
hoisted set + product + rescale at N = 2^16 replay bit-exactly against the
oracle, several times, with eager work and synchronizations between the
replays, and with new input data written into the captured input buffer."""
import numpy as np
import pytest

from oracle import boot as BT
from oracle import ckks
from tests import helpers as H
from tests import test_gpu_boot as GB
from tests import test_oracle_boot as TB

pytestmark = pytest.mark.gpu


def write_ct(buf, ct):
    import torch

    from paper_2510_03996_amd import he

    buf.data[:, : ct.level].copy_(he.to_device(ct.data, buf.data.device))
    torch.cuda.synchronize()


def test_captured_bootstrap_replays():
    import torch

    from paper_2510_03996_amd import he

    ctx, sk, pk, plan, keys, rk, cts, stc = TB.boot_setup(TB.BOOT_DA[1])
    pr = ctx.pr
    g = GB.boot_gpu_ctx()
    st = torch.cuda.Stream()
    try:
        GB.upload_boot_keys(g, keys, rk)
        g.layer_streams(2)
        desc = he.boot_desc(TB.BOOT_LEVELS, plan.degree, TB.BOOT_KMIN, pr.scale, double_angles=plan.double_angles)
        coeffs = list(plan.mod_coeffs(pr.q[0]))
        gcts = [g.pt_from_numpy(p.data, p.scale) for lv in cts for p in lv]
        gstc = [g.pt_from_numpy(p.data, p.scale) for lv in stc for p in lv]
        rng = np.random.default_rng(31)
        msgs = [rng.uniform(-1, 1, ctx.n // 2) for _ in range(3)]
        cins = [ctx.encrypt(pk, ctx.encode(v, pr.scale, 1), 31 + t) for t, v in enumerate(msgs)]
        wants = [BT.bootstrap(ctx, c, plan, keys, rk, cts, stc)[0] for c in cins]
        inbuf = g.ct_from_numpy(cins[0].data, cins[0].scale)
        out_e, out_g = g.new_ct(), g.new_ct()
        g.bootstrap(inbuf, desc, gcts, gstc, coeffs, out=out_e, stream=st)  # eager warm-up
        st.synchronize()
        H.assert_limbs_equal(out_e.numpy(), wants[0].data, "eager bootstrap")
        g.capture_begin(st)
        g.bootstrap(inbuf, desc, gcts, gstc, coeffs, out=out_g, stream=st)
        graph = g.capture_end(st)
        try:
            for rep, t in enumerate([0, 1, 1, 2]):
                write_ct(inbuf, cins[t])
                # eager work on the same stream between replays
                g.rotate_hoisted(g.ct_from_numpy(cins[0].data, cins[0].scale), [1, 2, 3], stream=st)
                graph.launch(st)
                st.synchronize()
                H.assert_limbs_equal(out_g.numpy(), wants[t].data, "replay %d (input %d)" % (rep, t))
                assert out_g.level == wants[t].level and out_g.scale == wants[t].scale
            dec = ctx.decrypt(sk, ckks.Ciphertext(out_g.numpy(), out_g.scale))
            assert np.max(np.abs(dec - msgs[2])) < TB.BOOT_TOL
        finally:
            graph.close()
    finally:
        g.close()


def test_captured_hoisted_set_n16():
    """Four rotations of one hoisted set (batched in one round, two helper
    streams at N = 2^16), a relinearized product and a rescale, captured and
    replayed three times with a new input each time."""
    import torch

    name = "config2"
    rs = [1, -1, 32, -1024]
    octx, _, _ = H.oracle_ctx(name)
    keys = H.oracle_keys(name, rs)
    rk = H.oracle_key(name, "relin")
    g = H.gpu_ctx(name)
    st = torch.cuda.Stream()
    try:
        from paper_2510_03996_amd import he

        for r in rs:
            g.key_upload(r, keys[r])
        g.key_upload(he.KEY_RELIN, rk)
        g.layer_streams(2)
        cins = [H.encrypt_slots(name, 70 + t, enc_id=t)[1] for t in range(3)]

        def want(ct):
            o = octx.rotate_hoisted(ct, rs, keys)
            return octx.rescale(octx.mul_relin(o[0], o[3], rk)), o

        inbuf = g.ct_from_numpy(cins[0].data, cins[0].scale)
        outs = [g.new_ct() for _ in rs]
        mid, prod = g.new_ct(), g.new_ct()

        def calls():  # every buffer allocated before the capture
            g.rotate_hoisted(inbuf, rs, outs=outs, stream=st)
            g.mul_relin(outs[0], outs[3], out=mid, stream=st)
            g.rescale(mid, out=prod, stream=st)

        calls()
        st.synchronize()
        w0, _ = want(cins[0])
        H.assert_limbs_equal(prod.numpy(), w0.data, "eager")
        g.capture_begin(st)
        calls()
        graph = g.capture_end(st)
        try:
            for t in (1, 2, 0):
                write_ct(inbuf, cins[t])
                graph.launch(st)
                st.synchronize()
                w, rot = want(cins[t])
                H.assert_limbs_equal(prod.numpy(), w.data, "replay, input %d" % t)
                for a, b in zip(outs, rot):
                    H.assert_limbs_equal(a.numpy(), b.data, "replayed rotation, input %d" % t)
        finally:
            graph.close()
    finally:
        g.close()


def test_capture_errors():
    import torch

    from paper_2510_03996_amd import he

    g = H.gpu_ctx("config0")
    try:
        with pytest.raises(he.HEError):
            g.capture_end(torch.cuda.Stream())  # not capturing
        # a key with a host copy cannot be loaded inside a capture
        octx, _, _ = H.oracle_ctx("config0")
        g.key_host_register(1, H.oracle_key("config0", 1))
        _, ct = H.encrypt_slots("config0", 5)
        gct = g.ct_from_numpy(ct.data, ct.scale)
        st = torch.cuda.Stream()
        out = g.new_ct()
        g.capture_begin(st)
        with pytest.raises(he.HEError, match="host copy"):
            g.rotate(gct, 1, out=out, stream=st)
        graph = g.capture_end(st)  # the capture itself ends cleanly
        graph.close()
    finally:
        g.close()


@pytest.mark.parametrize("name,n_streams", [("config1", 1), ("config2", 2)])
def test_captured_convolution_equals_eager(name, n_streams):
    """A captured he_conv2d (a 3x3, padding-1 convolution on a
    16x16 map of 4 channels, output channels over n_streams streams) replays bit-identically
    to the eager call, with a new input written between replays."""
    import torch

    import synth
    from paper_2510_03996_amd import he

    g = H.gpu_ctx(name)
    st = torch.cuda.Stream()
    try:
        g.layer_streams(n_streams)
        fm = he.fmap(4, 16, 16)
        pl = g.conv2d_plan(fm, 4, 3, 1, 1)
        for t, r in enumerate(pl.keys()):
            g.key_upload(r, synth.device_residues(900 + t, g.moduli, g.n, lead=(g.dnum, 2)))
        L = g.L
        sc = 2.0 ** 40
        kp = [he.Plaintext(b, sc) for b in synth.device_residues(950, g.moduli[:L], g.n, lead=(pl.n_kernel_pts,))]
        mp = [he.Plaintext(b, sc) for b in synth.device_residues(951, g.moduli[:L], g.n, lead=(max(1, pl.n_mask_pts),))]
        mp = mp[: pl.n_mask_pts]
        inputs = [synth.device_residues(960 + t, g.moduli[:L], g.n, lead=(2,)).contiguous() for t in range(2)]
        inbuf = he.Ciphertext(inputs[0].clone(), L, sc)
        ref = []
        for x in inputs:
            inbuf.data.copy_(x)
            o, _ = g.conv2d(inbuf, fm, 4, 3, 1, 1, kp, mp, stream=st)
            st.synchronize()
            ref.append(o.numpy())
        gout = g.new_ct()
        inbuf.data.copy_(inputs[0])
        g.conv2d(inbuf, fm, 4, 3, 1, 1, kp, mp, out=gout, stream=st)
        st.synchronize()
        g.capture_begin(st)
        g.conv2d(inbuf, fm, 4, 3, 1, 1, kp, mp, out=gout, stream=st)
        graph = g.capture_end(st)
        try:
            for t in (1, 0, 1):
                inbuf.data.copy_(inputs[t])
                torch.cuda.synchronize()
                graph.launch(st)
                st.synchronize()
                H.assert_limbs_equal(gout.numpy(), ref[t], "captured conv, input %d" % t)
        finally:
            graph.close()
    finally:
        g.close()


def test_bootstrap_capture_refused_at_n16():
    """he_bootstrap refuses graph capture at N = 2^16 (verified at N = 2^12
    only); the refusal comes before any work, and the capture ends cleanly."""
    import torch

    from paper_2510_03996_amd import he

    g = H.gpu_ctx("config2")
    st = torch.cuda.Stream()
    try:
        ct = g.new_ct(1)
        ct.level, ct.scale = 1, 2.0 ** 50
        out = g.new_ct()
        desc = he.boot_desc(3, 39, 12.0, 2.0 ** 50, double_angles=3)
        g.capture_begin(st)
        with pytest.raises(he.HEError, match="captured"):
            g.bootstrap(ct, desc, [], [], [0.0, 1.0], out=out, stream=st)
        g.capture_end(st).close()
    finally:
        g.close()
