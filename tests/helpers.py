"""Shared test setup: oracle contexts, keys and encrypted synthetic inputs.

Keys, ciphertexts and encoded plaintexts are produced by the oracle (the
client side of the paper's threat model) and uploaded to the GPU library,
which only ever sees ciphertexts, plaintexts and evaluation keys.
"""
import functools

import numpy as np

import synth
from oracle import ckks

SEED = 20251003


@functools.lru_cache(maxsize=None)
def oracle_ctx(name):
    pr = ckks.Params(**ckks.CONFIGS[name])
    ctx = ckks.Context(pr)
    sk, pk = ctx.keygen(SEED)
    return ctx, sk, pk


_keys = {}


def oracle_key(name, r):
    """Rotation key (r int) or relinearization key (r == 'relin'), cached."""
    ctx, sk, _ = oracle_ctx(name)
    k = (name, r)
    if k not in _keys:
        _keys[k] = ctx.gen_relin_key(sk, SEED) if r == "relin" else ctx.gen_rotation_key(sk, r, SEED)
    return _keys[k]


def oracle_keys(name, rs):
    return {r: oracle_key(name, r) for r in rs}


def encrypt_slots(name, seed, level=None, enc_id=0, values=None):
    ctx, sk, pk = oracle_ctx(name)
    pr = ctx.pr
    v = synth.uniform_slots(seed, pr.n // 2) if values is None else values
    ct = ctx.encrypt(pk, ctx.encode(v, pr.scale, pr.L), SEED + seed, enc_id)
    if level is not None and level < ct.level:
        ct = ctx.drop_level(ct, level)
    return v, ct


def encode_slots(name, seed, level, scale=None):
    ctx, _, _ = oracle_ctx(name)
    v = synth.uniform_slots(seed, ctx.pr.n // 2, stream=9)
    return v, ctx.encode(v, scale or ctx.pr.scale, level)


def gpu_ctx(name):
    """A GPU library context for a configuration (primes chosen by the library)."""
    from paper_2510_03996_amd import he

    cfg = ckks.CONFIGS[name]
    return he.Context(cfg["log_n"], cfg["q_bits"], cfg["p_bits"], cfg["alpha"])


def assert_limbs_equal(got, want, what=""):
    got = np.asarray(got, dtype=np.uint64)
    want = np.asarray(want, dtype=np.uint64)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    bad = np.argwhere(got != want)
    assert bad.size == 0, "%s: %d mismatching residues, first at %s" % (what, len(bad), bad[:3].tolist())
