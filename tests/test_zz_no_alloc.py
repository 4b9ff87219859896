"""he_rotate_noalloc (key-switch workspace in the library's static device
array, nothing allocated) against he_rotate on the same inputs: bit-identical
ciphertexts on two calls in a row, the second with a smaller input (lower
level, other key), at N = 2^16 (the headline ring) and N = 2^14."""
import pytest
import torch

import synth

CFG2 = dict(log_n=16, q_bits=[60] + [50] * 23, p_bits=[50] * 9, alpha=8)
CFG1 = dict(log_n=14, q_bits=[60] + [45] * 7, p_bits=[60, 60], alpha=2)


def _ctx(cfg):
    from paper_2510_03996_amd import he

    return he.Context(cfg["log_n"], cfg["q_bits"], cfg["p_bits"], cfg["alpha"])


def _ct(ctx, level, seed):
    from paper_2510_03996_amd import he

    d = synth.device_residues(seed, ctx.moduli[:level], ctx.n, lead=(2,))
    return he.Ciphertext(d.contiguous(), level, 2.0 ** 40)


@pytest.mark.gpu
@pytest.mark.parametrize("cfg,calls", [(CFG2, [(24, 1), (13, -5)]), (CFG1, [(8, 3), (3, -1)])],
                         ids=["n16", "n14"])
def test_rotate_noalloc_matches_rotate(cfg, calls):
    print("noalloc: log_n", cfg["log_n"], "calls", calls, flush=True)
    ctx = _ctx(cfg)
    keys = sorted({r for _, r in calls})
    for t, r in enumerate(keys):
        ctx.key_upload(r, synth.device_residues(700 + t, ctx.moduli, ctx.n, lead=(ctx.dnum, 2)))
    stream = torch.cuda.Stream()  # a stream without a lane: nothing may be allocated for it
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    outs = []
    for i, (level, r) in enumerate(calls):
        ct = _ct(ctx, level, 800 + i)
        out = ctx.new_ct(level)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            ctx.rotate_noalloc(ct, r, out, stream=stream)
        stream.synchronize()
        outs.append((ct, r, out))
    free1 = torch.cuda.mem_get_info()[0]
    # a lane for the stream would take its key-switch workspace (tens of MB)
    assert free0 - free1 < (8 << 20), (free0, free1)
    for ct, r, out in outs:
        ref = ctx.rotate(ct, r)
        torch.cuda.synchronize()
        assert out.level == ref.level and out.scale == ref.scale
        assert torch.equal(out.data[:, :out.level], ref.data[:, :ref.level])
    ctx.close()


@pytest.mark.gpu
def test_rotate_noalloc_rejects_host_backed_keys():
    from paper_2510_03996_amd import he

    ctx = _ctx(CFG1)
    k = synth.device_residues(710, ctx.moduli, ctx.n, lead=(ctx.dnum, 2))
    ctx.key_host_register(2, k.cpu().numpy().view("uint64"))
    ct = _ct(ctx, 8, 811)
    out = ctx.new_ct(8)
    with pytest.raises(he.HEError):
        ctx.rotate_noalloc(ct, 2, out)
    ctx.close()
