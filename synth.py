"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds none of the CKKS arithmetic: it only draws numbers (slot
vectors, images, weights, rotation sets, arrival times, raw residues) from
seeded numpy generators, with the shapes and distributions of the workloads
the paper evaluates (MNIST-shaped 1x28x28 and CIFAR-shaped 16x32x32 feature
maps, LeNet-5 / ResNet-20 layer weights).  Both the GPU path and the CPU
oracle consume what it returns; neither is imported here.
"""
import numpy as np


def rng(seed, stream=0):
    return np.random.default_rng([int(seed), int(stream)])


def uniform_slots(seed, n, lo=-1.0, hi=1.0, stream=0):
    """n values uniform in [lo, hi)."""
    return rng(seed, stream).uniform(lo, hi, n)


def image(seed, c, h, w, stream=1):
    """A C x H x W input tensor, uniform [-1, 1] (stand-in for a normalised image)."""
    return rng(seed, stream).uniform(-1.0, 1.0, (c, h, w))


def conv_weights(seed, f, c, k, sigma, stream=2):
    """F x C x k x k kernel weights ~ N(0, sigma^2)."""
    return rng(seed, stream).normal(0.0, sigma, (f, c, k, k))


def fc_weights(seed, m, n, sigma, stream=3):
    return rng(seed, stream).normal(0.0, sigma, (m, n))


def residues(seed, moduli, n, stream=4):
    """uint64 [len(moduli)][n], limb i uniform in [0, moduli[i]) — a stand-in
    for ciphertext / key / plaintext limbs (RLWE samples look uniform)."""
    g = rng(seed, stream)
    return np.stack([g.integers(0, int(q), n, dtype=np.uint64) for q in moduli])


def rotation_sets(seed, n_ct, pool, n_lo, n_hi, m_lo, m_hi, stream=5):
    """Per ciphertext: a set of n ~ U{n_lo..n_hi} distinct rotation amounts
    drawn from `pool` by seeded shuffle, and an output count m ~ U{m_lo..m_hi}."""
    g = rng(seed, stream)
    sets, outs = [], []
    for _ in range(n_ct):
        n = int(g.integers(n_lo, n_hi + 1))
        sets.append([int(x) for x in g.permutation(np.asarray(pool))[:n]])
        outs.append(int(g.integers(m_lo, m_hi + 1)))
    return sets, outs


def poisson_arrivals(seed, rate, count, stream=6):
    """Arrival times (s) of a Poisson process with the given rate."""
    return np.cumsum(rng(seed, stream).exponential(1.0 / rate, count))


def request_mix(seed, count, p_small=0.75, stream=7):
    """Request kinds: 0 (small ring) with probability p_small, else 1."""
    return (rng(seed, stream).uniform(0, 1, count) >= p_small).astype(np.int64)


def device_residues(seed, moduli, n, lead=(), device="cuda"):
    """int64 torch tensor [*lead][len(moduli)][n] on `device`, limb i uniform in
    [0, moduli[i]) — large seeded stand-ins for keys / ciphertexts /
    plaintexts generated directly in device memory."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    out = torch.empty(tuple(lead) + (len(moduli), n), dtype=torch.int64, device=device)
    for i, q in enumerate(moduli):
        out[..., i, :] = torch.randint(0, int(q), tuple(lead) + (n,), generator=g, dtype=torch.int64, device=device)
    return out
