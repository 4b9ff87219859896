"""Loader for the oracle's C routines (test infrastructure only).

Builds ``oracle/liboracle.so`` from ``oracle/oracle.c`` with gcc when it is
missing, then exposes thin numpy-array wrappers.  The oracle never loads the
GPU library and the GPU library never loads this one.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(force=False):
    """Compile the oracle C code (plain gcc, OpenMP, no fp contraction)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


_lib = None
u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        c_u64, c_int, c_sz = ctypes.c_uint64, ctypes.c_int, ctypes.c_size_t
        L.or_powmod.restype = c_u64
        L.or_powmod.argtypes = [c_u64, c_u64, c_u64]
        L.or_invmod.restype = c_u64
        L.or_invmod.argtypes = [c_u64, c_u64]
        L.or_is_prime.restype = c_int
        L.or_is_prime.argtypes = [c_u64]
        L.or_ntt.argtypes = [u64p, c_int, c_sz, u64p, u64p, c_int]
        for f in ("or_mul", "or_add", "or_sub", "or_mul_scalar"):
            getattr(L, f).argtypes = [u64p, u64p, u64p, c_int, c_sz, u64p]
        L.or_reduce_row.argtypes = [u64p, u64p, c_int, c_sz, u64p]
        L.or_from_signed.argtypes = [i64p, u64p, c_int, c_sz, u64p]
        L.or_bconv.argtypes = [u64p, c_int, u64p, u64p, u64p, c_int, u64p, u64p, c_sz]
        L.or_automorph_coeff.argtypes = [u64p, u64p, c_int, c_sz, u64p, c_u64]
        L.or_automorph_perm.argtypes = [c_sz, c_u64, i64p]
        L.or_sample_uniform.argtypes = [c_u64, c_u64, u64p, c_int, c_sz, u64p]
        L.or_sample_ternary.argtypes = [c_u64, c_u64, c_sz, i64p]
        L.or_sample_gaussian.argtypes = [c_u64, c_u64, c_sz, ctypes.c_double, ctypes.c_int64, i64p]
        L.or_rng_first.restype = c_u64
        L.or_rng_first.argtypes = [c_u64, c_u64]
        _lib = L
    return _lib


def _u64(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


def ntt(a, moduli, psis, inverse=False):
    """In-place copy semantics: returns the (inverse) negacyclic NTT of each limb."""
    a = _u64(a).copy()
    nl, n = a.shape
    lib().or_ntt(a, nl, n, _u64(moduli), _u64(psis), 1 if inverse else 0)
    return a


def _binop(name, a, b, moduli):
    a, b = _u64(a), _u64(b)
    out = np.empty_like(a)
    nl, n = a.shape
    getattr(lib(), name)(a, b, out, nl, n, _u64(moduli))
    return out


def mul(a, b, moduli):
    return _binop("or_mul", a, b, moduli)


def add(a, b, moduli):
    return _binop("or_add", a, b, moduli)


def sub(a, b, moduli):
    return _binop("or_sub", a, b, moduli)


def mul_scalar(a, consts, moduli):
    a = _u64(a)
    out = np.empty_like(a)
    nl, n = a.shape
    lib().or_mul_scalar(a, _u64(consts), out, nl, n, _u64(moduli))
    return out


def reduce_row(row, moduli):
    row = _u64(row)
    out = np.empty((len(moduli), row.shape[0]), dtype=np.uint64)
    lib().or_reduce_row(row, out, len(moduli), row.shape[0], _u64(moduli))
    return out


def from_signed(s, moduli):
    s = np.ascontiguousarray(s, dtype=np.int64)
    out = np.empty((len(moduli), s.shape[0]), dtype=np.uint64)
    lib().or_from_signed(s, out, len(moduli), s.shape[0], _u64(moduli))
    return out


def bconv(x, qin, qhat_inv, qout, qhat):
    x = _u64(x)
    nin, n = x.shape
    y = np.empty((len(qout), n), dtype=np.uint64)
    lib().or_bconv(x, nin, _u64(qin), _u64(qhat_inv), y, len(qout), _u64(qout), _u64(qhat), n)
    return y


def automorph_coeff(a, moduli, g):
    a = _u64(a)
    out = np.empty_like(a)
    nl, n = a.shape
    lib().or_automorph_coeff(a, out, nl, n, _u64(moduli), g)
    return out


def automorph_perm(n, g):
    perm = np.empty(n, dtype=np.int64)
    lib().or_automorph_perm(n, g, perm)
    return perm


def sample_uniform(seed, stream, moduli, n):
    out = np.empty((len(moduli), n), dtype=np.uint64)
    lib().or_sample_uniform(seed, stream, _u64(moduli), len(moduli), n, out)
    return out


def sample_ternary(seed, stream, n):
    out = np.empty(n, dtype=np.int64)
    lib().or_sample_ternary(seed, stream, n, out)
    return out


def sample_gaussian(seed, stream, n, sigma=3.2, bound=19):
    out = np.empty(n, dtype=np.int64)
    lib().or_sample_gaussian(seed, stream, n, sigma, bound, out)
    return out


def is_prime(x):
    return bool(lib().or_is_prime(x))
