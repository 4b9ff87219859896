"""RNS-CKKS oracle — TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct CPU definition of the CKKS arithmetic under
FHEON's encrypted CNN layers.  The paper takes RNS-CKKS over
R = Z[X]/(X^N + 1) from its CPU library (Background, "CKKS scheme") and names
hoisted "fast rotations"; it does not write down the ring arithmetic.  This
module therefore writes out the standard RNS-CKKS definitions with every
convention pinned (prime choice, NTT order, digit split, floor-type basis
conversion, rescale, key layout), so that a GPU implementation can be held to
the same integers bit for bit.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It imports nothing from the GPU package.

Layout conventions (shared *by specification*, not by code, with the GPU side):
  * a polynomial over a basis is a uint64 array [limbs][N]; every limb is in
    NTT form (see ``oracle.c``: bit-reversed evaluation at odd powers of the
    minimum primitive 2N-th root psi);
  * a ciphertext is uint64 [2][l][N] (c0, c1) at level l = number of active
    Q limbs, plus a float64 scale;
  * an evaluation (key-switching) key is uint64 [dnum][2][L+K][N]: for digit j,
    poly 0 is b_j and poly 1 is a_j, limbs q_0..q_{L-1} then p_0..p_{K-1}.

Parity status: every function below is pinned by the tests in
``tests/test_oracle_*.py`` (brute force on tiny rings with Python integers,
closed-form identities, decryption identities, FP64 references).
"""
import math

import numpy as np

from . import _lib as C

RELIN = "relin"
# key id of the conjugation key (Galois element 2N - 1: every slot is
# replaced by its complex conjugate); bootstrapping needs it to split the
# real and imaginary parts of a coefficient-to-slot result
CONJ = "conj"


# --------------------------------------------------------------------- primes
def gen_primes(log_n, q_bits, p_bits):
    """Prime selection rule (the paper only fixes bit sizes).

    For a bit size b, candidates are q = k*2N + 1 < 2^b in descending k,
    accepted when prime and q > 2^(b-1).  Allocation order: q_0, then
    q_1..q_{L-1}, then the special primes, each taking the largest not yet
    taken prime of its size.
    """
    two_n = 2 << log_n
    taken = set()
    nxt = {}

    def take(b):
        k = nxt.get(b, ((1 << b) - 2) // two_n)
        while True:
            q = k * two_n + 1
            if q <= (1 << (b - 1)):
                raise ValueError("ran out of %d-bit primes" % b)
            k -= 1
            if q < (1 << b) and q not in taken and C.is_prime(q):
                taken.add(q)
                nxt[b] = k
                return q

    qs = [take(b) for b in q_bits]
    ps = [take(b) for b in p_bits]
    return qs, ps


def min_root(q, n):
    """psi = the minimum primitive 2N-th root of unity modulo q."""
    two_n = 2 * n
    assert (q - 1) % two_n == 0
    x = 2
    while True:
        cand = pow(x, (q - 1) // two_n, q)
        if pow(cand, n, q) == q - 1:
            break
        x += 1
    sq = cand * cand % q
    best, cur = cand, cand
    for _ in range(n - 1):
        cur = cur * sq % q
        if cur < best:
            best = cur
    return best


def sparse_ternary(seed, stream, n, h):
    """Ternary secret with exactly h nonzero coefficients: positions are the
    first h distinct values of a stream of uniform draws modulo n, signs a
    second stream of uniform bits (1 -> +1, 0 -> -1).  Both streams come from
    the seeded generator the rest of the sampling uses."""
    draws = C.sample_uniform(seed, stream, [n], 8 * h + 64)[0]
    pos, seen = [], set()
    for d in draws:
        d = int(d)
        if d not in seen:
            seen.add(d)
            pos.append(d)
            if len(pos) == h:
                break
    if len(pos) != h:
        raise ValueError("hamming weight too large for the ring")
    bits = C.sample_uniform(seed, stream + 1, [2], h)[0]
    s = np.zeros(n, dtype=np.int64)
    s[pos] = np.where(bits == 1, 1, -1)
    return s


# --------------------------------------------------------------------- params
class Params:
    """CKKS parameters: ring degree 2^log_n, Q primes, special primes P,
    alpha = Q limbs per key-switching digit, default scale 2^log_scale."""

    def __init__(self, log_n, q_bits, p_bits, alpha, log_scale, primes=None):
        self.log_n = log_n
        self.n = 1 << log_n
        self.alpha = alpha
        self.log_scale = log_scale
        self.scale = float(2.0 ** log_scale)
        if primes is None:
            self.q, self.p = gen_primes(log_n, q_bits, p_bits)
        else:
            self.q, self.p = list(primes[0]), list(primes[1])
        self.L = len(self.q)
        self.K = len(self.p)
        self.moduli = self.q + self.p
        self.psi = [min_root(m, self.n) for m in self.moduli]
        self.P = math.prod(self.p)

    def dnum(self, level):
        return -(-level // self.alpha)

    def digit(self, j, level):
        return list(range(j * self.alpha, min((j + 1) * self.alpha, level)))


CONFIGS = {
    # tiny conv: N=2^12, one 54-bit + two 40-bit Q primes, one 55-bit P prime,
    # one limb per digit, scale 2^40
    "config0": dict(log_n=12, q_bits=[54, 40, 40], p_bits=[55], alpha=1, log_scale=40),
    # LeNet-5-shaped: N=2^14, one 60-bit + seven 45-bit, two 60-bit P primes,
    # dnum=4 (two limbs per digit), scale 2^45
    "config1": dict(log_n=14, q_bits=[60] + [45] * 7, p_bits=[60, 60], alpha=2, log_scale=45),
    # ResNet-20-shaped: N=2^16, one 60-bit + 23 50-bit, nine 50-bit P primes
    # (P = 2^450 above the largest digit, 2^410), dnum=3 (eight limbs per
    # digit), scale 2^50
    "config2": dict(log_n=16, q_bits=[60] + [50] * 23, p_bits=[50] * 9, alpha=8, log_scale=50),
}


# --------------------------------------------------------------------- objects
class Ciphertext:
    def __init__(self, data, scale):
        self.data = np.ascontiguousarray(data, dtype=np.uint64)
        assert self.data.ndim == 3 and self.data.shape[0] == 2
        self.scale = float(scale)

    @property
    def level(self):
        return self.data.shape[1]

    def copy(self):
        return Ciphertext(self.data.copy(), self.scale)


class Plaintext:
    def __init__(self, data, scale):
        self.data = np.ascontiguousarray(data, dtype=np.uint64)
        self.scale = float(scale)

    @property
    def level(self):
        return self.data.shape[0]


class SecretKey:
    def __init__(self, s, s_ntt):
        self.s = s            # int64 [N], ternary coefficients
        self.s_ntt = s_ntt    # uint64 [L+K][N]


class PublicKey:
    def __init__(self, b, a):
        self.b, self.a = b, a  # uint64 [L][N] each


class Context:
    """All CKKS operations of the oracle for one parameter set."""

    def __init__(self, params):
        self.pr = params
        self.n = params.n
        self._perm_cache = {}
        self._modup_cache = {}
        self._moddown_cache = {}

    # ---- basis helpers
    def qs(self, level):
        return self.pr.q[:level]

    def psis(self, level):
        return self.pr.psi[:level]

    def ext_moduli(self, level):
        return self.pr.q[:level] + self.pr.p

    def ext_psis(self, level):
        return self.pr.psi[:level] + self.pr.psi[self.pr.L:]

    def ntt(self, a, moduli, psis):
        return C.ntt(a, moduli, psis, inverse=False)

    def intt(self, a, moduli, psis):
        return C.ntt(a, moduli, psis, inverse=True)

    # ---- encoding (client side; canonical embedding, N/2 real slots)
    def slot_exponents(self):
        """e_j = 5^j mod 2N: slot j is the evaluation at zeta^(e_j), zeta = exp(i pi / N)."""
        n2 = 2 * self.n
        e = np.empty(self.n // 2, dtype=np.int64)
        cur = 1
        for j in range(self.n // 2):
            e[j] = cur
            cur = cur * 5 % n2
        return e

    def encode_coeffs(self, values, scale):
        """Real slot vector -> integer coefficients llround(scale * m_k), where
        m_k = (2/N) sum_j v_j cos(pi 5^j k / N), the inverse canonical
        embedding of a conjugate-symmetric vector.  Computed with one
        length-2N FFT (z placed at exponents 5^j and -5^j)."""
        n = self.n
        v = np.zeros(n // 2, dtype=np.float64)
        vals = np.asarray(values, dtype=np.float64).ravel()
        assert vals.size <= n // 2
        v[: vals.size] = vals
        e = self.slot_exponents()
        z = np.zeros(2 * n, dtype=np.complex128)
        z[e] = v
        z[(2 * n - e) % (2 * n)] = v
        m = np.fft.fft(z)[:n].real / n
        x = m * scale
        r = np.where(x >= 0, np.floor(x + 0.5), -np.floor(-x + 0.5))
        assert np.all(np.abs(r) < 2.0 ** 62)
        return r.astype(np.int64)

    def encode_coeffs_complex(self, values, scale):
        """Complex slot vector z (N/2 slots) -> integer coefficients
        llround(scale * m_k), m_k = (2/N) Re(sum_j z_j zeta^(-5^j k)): the
        inverse canonical embedding of (z, conj(z)) at the exponents
        (5^j, -5^j).  For real z this is encode_coeffs."""
        n = self.n
        v = np.zeros(n // 2, dtype=np.complex128)
        vals = np.asarray(values, dtype=np.complex128).ravel()
        assert vals.size <= n // 2
        v[: vals.size] = vals
        e = self.slot_exponents()
        z = np.zeros(2 * n, dtype=np.complex128)
        z[e] = v
        z[(2 * n - e) % (2 * n)] = np.conj(v)
        m = np.fft.fft(z)[:n].real / n
        x = m * scale
        r = np.where(x >= 0, np.floor(x + 0.5), -np.floor(-x + 0.5))
        assert np.all(np.abs(r) < 2.0 ** 62)
        return r.astype(np.int64)

    def encode_complex(self, values, scale, level):
        """encode() for a complex slot vector."""
        coeffs = self.encode_coeffs_complex(values, scale)
        rns = C.from_signed(coeffs, self.qs(level))
        return Plaintext(self.ntt(rns, self.qs(level), self.psis(level)), scale)

    def decode_coeffs_complex(self, m, scale):
        """Integer (float64) coefficients -> complex slot values
        z_j = sum_k m_k zeta^(5^j k) / scale."""
        n = self.n
        pad = np.zeros(2 * n, dtype=np.complex128)
        pad[:n] = m
        w = np.fft.ifft(pad) * (2 * n)
        return w[self.slot_exponents()] / scale

    def decrypt_complex(self, sk, ct):
        return self.decode_coeffs_complex(self.decrypt_coeffs(sk, ct), ct.scale)

    def encode(self, values, scale, level):
        """Encode to an RNS plaintext in NTT form over q_0..q_{level-1}."""
        coeffs = self.encode_coeffs(values, scale)
        rns = C.from_signed(coeffs, self.qs(level))
        return Plaintext(self.ntt(rns, self.qs(level), self.psis(level)), scale)

    def encode_const(self, c, scale, level):
        """A constant encodes to the constant polynomial llround(c*scale);
        its NTT form holds that value in every position."""
        x = c * scale
        r = int(math.floor(x + 0.5)) if x >= 0 else -int(math.floor(-x + 0.5))
        poly = np.zeros(self.n, dtype=np.int64)
        poly[0] = r
        coeff = C.from_signed(poly, self.qs(level))
        return Plaintext(self.ntt(coeff, self.qs(level), self.psis(level)), scale)

    def decode_coeffs(self, m, scale):
        """Integer (float64) coefficients -> real slot values:
        v_j = Re(sum_k m_k zeta^(5^j k)) / scale."""
        n = self.n
        pad = np.zeros(2 * n, dtype=np.complex128)
        pad[:n] = m
        w = np.fft.ifft(pad) * (2 * n)
        return w[self.slot_exponents()].real / scale

    # ---- keys (client side)
    def keygen(self, seed, hamming=0):
        """Secret, public key.  hamming = 0: uniform ternary secret; else a
        sparse ternary secret with exactly `hamming` nonzero coefficients
        (bootstrapping's choice: it bounds the multiple of q_0 that ModRaise
        adds, see ``sparse_ternary``)."""
        pr = self.pr
        s = sparse_ternary(seed, 1, self.n, hamming) if hamming else C.sample_ternary(seed, 1, self.n)
        s_ntt = self.ntt(C.from_signed(s, pr.moduli), pr.moduli, pr.psi)
        sk = SecretKey(s, s_ntt)
        a = C.sample_uniform(seed, 2, pr.q, self.n)
        e = self.ntt(C.from_signed(C.sample_gaussian(seed, 3, self.n), pr.q), pr.q, pr.psi[: pr.L])
        b = C.sub(e, C.mul(a, s_ntt[: pr.L], pr.q), pr.q)
        return sk, PublicKey(b, a)

    def gen_switch_key(self, sk, s_prime_q, seed, stream):
        """Hybrid key-switching key from s' to s (gadget P * Qhat_j * [Qhat_j^-1]_{Q_j}).

        For digit j over Q_L u P:  a_j uniform, e_j rounded Gaussian,
          b_j = -a_j s + e_j + [P]_{q_i} s'   on the limbs q_i of digit j,
          b_j = -a_j s + e_j                  on every other limb (P included).
        s_prime_q: s' in NTT form over q_0..q_{L-1}.  Returns [dnum][2][L+K][N].
        """
        pr = self.pr
        mods = pr.moduli
        dnum = pr.dnum(pr.L)
        key = np.empty((dnum, 2, pr.L + pr.K, self.n), dtype=np.uint64)
        for j in range(dnum):
            st = stream * 64 + j
            a = C.sample_uniform(seed, 1_000_000 + st, mods, self.n)
            e = C.from_signed(C.sample_gaussian(seed, 2_000_000 + st, self.n), mods)
            e = self.ntt(e, mods, pr.psi)
            b = C.sub(e, C.mul(a, sk.s_ntt, mods), mods)
            for i in pr.digit(j, pr.L):
                gadget = C.mul_scalar(s_prime_q[i:i + 1], [pr.P % pr.q[i]], [pr.q[i]])
                b[i:i + 1] = C.add(b[i:i + 1], gadget, [pr.q[i]])
            key[j, 0] = b
            key[j, 1] = a
        return key

    def galois_element(self, r):
        """Rot_r (slot i <- slot i + r) is X -> X^g with g = 5^(r mod N/2) mod 2N;
        the conjugation (r = CONJ) is X -> X^(2N-1)."""
        if r == CONJ:
            return 2 * self.n - 1
        return pow(5, r % (self.n // 2), 2 * self.n)

    def gen_rotation_key(self, sk, r, seed):
        """Key switching from phi_g(s) to s for Rot_r, or for the conjugation
        when r = CONJ (its sampling stream follows every rotation's)."""
        g = self.galois_element(r)
        s_rot = sk.s_ntt[: self.pr.L][:, self.perm(g)]
        stream = 10 + (self.n // 2 if r == CONJ else r % (self.n // 2))
        return self.gen_switch_key(sk, s_rot, seed, stream)

    def gen_relin_key(self, sk, seed):
        sq = C.mul(sk.s_ntt[: self.pr.L], sk.s_ntt[: self.pr.L], self.pr.q)
        return self.gen_switch_key(sk, sq, seed, 5)

    # ---- encryption / decryption (client side)
    def encrypt(self, pk, pt, seed, enc_id=0):
        """Public-key encryption at the plaintext's level:
        (v b + e0 + m, v a + e1), v ternary, e0, e1 rounded Gaussian."""
        level = pt.level
        qs, ps = self.qs(level), self.psis(level)
        st = 100 + 3 * enc_id
        v = self.ntt(C.from_signed(C.sample_ternary(seed, st, self.n), qs), qs, ps)
        e0 = self.ntt(C.from_signed(C.sample_gaussian(seed, st + 1, self.n), qs), qs, ps)
        e1 = self.ntt(C.from_signed(C.sample_gaussian(seed, st + 2, self.n), qs), qs, ps)
        c0 = C.add(C.add(C.mul(v, pk.b[:level], qs), e0, qs), pt.data[:level], qs)
        c1 = C.add(C.mul(v, pk.a[:level], qs), e1, qs)
        return Ciphertext(np.stack([c0, c1]), pt.scale)

    def decrypt_coeffs(self, sk, ct):
        """m = c0 + c1 s modulo q_0 only, centred (valid while |m| < q_0/2)."""
        q0 = [self.pr.q[0]]
        m = C.add(ct.data[0, :1], C.mul(ct.data[1, :1], sk.s_ntt[:1], q0), q0)
        m = self.intt(m, q0, self.pr.psi[:1])[0]
        q = self.pr.q[0]
        return np.where(m > q // 2, -(q - m).astype(np.float64), m.astype(np.float64))

    def decrypt(self, sk, ct):
        return self.decode_coeffs(self.decrypt_coeffs(sk, ct), ct.scale)

    # ---- exact ring operations (server side)
    def _check_pair(self, a, b):
        if a.level != b.level:
            raise ValueError("level mismatch")
        if a.scale != b.scale:
            raise ValueError("scale mismatch")

    def add(self, a, b):
        self._check_pair(a, b)
        qs = self.qs(a.level)
        return Ciphertext(np.stack([C.add(a.data[k], b.data[k], qs) for k in range(2)]), a.scale)

    def sub(self, a, b):
        self._check_pair(a, b)
        qs = self.qs(a.level)
        return Ciphertext(np.stack([C.sub(a.data[k], b.data[k], qs) for k in range(2)]), a.scale)

    def add_plain(self, a, pt):
        if a.scale != pt.scale:
            raise ValueError("scale mismatch")
        qs = self.qs(a.level)
        return Ciphertext(np.stack([C.add(a.data[0], pt.data[: a.level], qs), a.data[1]]), a.scale)

    def mul_plain(self, a, pt):
        """ct (.) pt per limb at the ciphertext's level; scales multiply."""
        qs = self.qs(a.level)
        d = np.stack([C.mul(a.data[k], pt.data[: a.level], qs) for k in range(2)])
        return Ciphertext(d, a.scale * pt.scale)

    def drop_level(self, a, level):
        """Level alignment: keep limbs q_0..q_{level-1}; no scale change."""
        assert level <= a.level
        return Ciphertext(a.data[:, :level].copy(), a.scale)

    def rescale(self, a):
        """Floor rescale by the top prime q_t (t = level-1):
        r = [c]_{q_t} in [0, q_t) (coefficient form), then
        c'_i = (c_i - (r mod q_i)) * q_t^{-1} mod q_i  for i < t.
        Equals floor(c / q_t) as integers; scale / q_t."""
        t = a.level - 1
        qt = self.pr.q[t]
        qs, ps = self.qs(t), self.psis(t)
        out = np.empty((2, t, self.n), dtype=np.uint64)
        for k in range(2):
            r = self.intt(a.data[k, t:t + 1], [qt], [self.pr.psi[t]])[0]
            r_ntt = self.ntt(C.reduce_row(r, qs), qs, ps)
            diff = C.sub(a.data[k, :t], r_ntt, qs)
            out[k] = C.mul_scalar(diff, [pow(qt, -1, q) for q in qs], qs)
        return Ciphertext(out, a.scale / float(qt))

    # ---- key switching
    def perm(self, g):
        if g not in self._perm_cache:
            self._perm_cache[g] = C.automorph_perm(self.n, g)
        return self._perm_cache[g]

    def automorph(self, poly, g):
        """phi_g on NTT-form limbs (index map)."""
        if g == 1:
            return poly.copy()
        return np.ascontiguousarray(poly[:, self.perm(g)])

    def modup_consts(self, j, level):
        key = (j, level)
        if key not in self._modup_cache:
            pr = self.pr
            idx = pr.digit(j, level)
            qin = [pr.q[i] for i in idx]
            Qj = math.prod(qin)
            outs = [i for i in range(level) if i not in idx]
            qout = [pr.q[i] for i in outs] + pr.p
            qhat_inv = [pow(Qj // qi, -1, qi) for qi in qin]
            qhat = [[(Qj // qi) % po for po in qout] for qi in qin]
            self._modup_cache[key] = (idx, outs, qin, qout, qhat_inv, np.array(qhat, dtype=np.uint64).ravel())
        return self._modup_cache[key]

    def modup(self, c1, level):
        """Digit decomposition + basis extension of an NTT-form poly over Q_l.

        Digit j = limbs of Q_j (alpha consecutive limbs, the last one possibly
        shorter).  Returns dnum arrays over Q_l u P (NTT form): the digit's own
        limbs are copied; every other limb is the floor-type basis conversion
        of the digit's coefficients, then NTT."""
        pr = self.pr
        coeff = self.intt(c1, self.qs(level), self.psis(level))
        emods, epsis = self.ext_moduli(level), self.ext_psis(level)
        out = []
        for j in range(pr.dnum(level)):
            idx, outs, qin, qout, qhat_inv, qhat = self.modup_consts(j, level)
            ext = np.empty((level + pr.K, self.n), dtype=np.uint64)
            ext[idx] = c1[idx]
            y = C.bconv(coeff[idx], qin, qhat_inv, qout, qhat)
            pos = outs + list(range(level, level + pr.K))
            y = self.ntt(y, [emods[i] for i in pos], [epsis[i] for i in pos])
            ext[pos] = y
            out.append(ext)
        return out

    def moddown_consts(self, level):
        if level not in self._moddown_cache:
            pr = self.pr
            P = pr.P
            qhat_inv = [pow(P // p, -1, p) for p in pr.p]
            qhat = [[(P // p) % q for q in pr.q[:level]] for p in pr.p]
            pinv = [pow(P % q, -1, q) for q in pr.q[:level]]
            self._moddown_cache[level] = (qhat_inv, np.array(qhat, dtype=np.uint64).ravel(), pinv)
        return self._moddown_cache[level]

    def moddown(self, u, level):
        """(u - BConv_{P->Q}([u]_P)) * P^{-1} mod q_i  (floor type), NTT form in and out."""
        pr = self.pr
        qhat_inv, qhat, pinv = self.moddown_consts(level)
        up = self.intt(u[level:], pr.p, pr.psi[pr.L:])
        y = C.bconv(up, pr.p, qhat_inv, self.qs(level), qhat)
        y = self.ntt(y, self.qs(level), self.psis(level))
        return C.mul_scalar(C.sub(u[:level], y, self.qs(level)), pinv, self.qs(level))

    def key_limbs(self, key, level):
        """The key restricted to the active limbs q_0..q_{l-1} and all of P."""
        L = self.pr.L
        sel = list(range(level)) + list(range(L, L + self.pr.K))
        return key[:, :, sel]

    def keyswitch_ext(self, ext, key, g, level):
        """Inner product of the (automorphed) extended digits with the key,
        then ModDown of both accumulators."""
        emods = self.ext_moduli(level)
        k = self.key_limbs(key, level)
        u0 = np.zeros((level + self.pr.K, self.n), dtype=np.uint64)
        u1 = np.zeros_like(u0)
        for j, d in enumerate(ext):
            dg = self.automorph(d, g)
            u0 = C.add(u0, C.mul(dg, k[j, 0], emods), emods)
            u1 = C.add(u1, C.mul(dg, k[j, 1], emods), emods)
        return self.moddown(u0, level), self.moddown(u1, level)

    def rotate_hoisted(self, ct, rs, keys):
        """Hoisted rotations: one ModUp of c1, then for every r:
        out_r = (phi_g(c0) + u0, u1) with (u0, u1) = ModDown(<phi_g(ModUp(c1)), evk_r>).
        ``keys`` maps r -> key array.  Rot_0 returns a copy (no key switch)."""
        level = ct.level
        qs = self.qs(level)
        ext = None
        outs = []
        for r in rs:
            g = self.galois_element(r)
            if g == 1:
                outs.append(ct.copy())
                continue
            if ext is None:
                ext = self.modup(ct.data[1], level)
            u0, u1 = self.keyswitch_ext(ext, keys[r], g, level)
            c0 = C.add(self.automorph(ct.data[0], g), u0, qs)
            outs.append(Ciphertext(np.stack([c0, u1]), ct.scale))
        return outs

    def rotate(self, ct, r, keys):
        return self.rotate_hoisted(ct, [r], keys)[0]

    def tensor(self, a, b):
        """(a0 b0, a0 b1 + a1 b0, a1 b1) at a common level; scales multiply."""
        self._check_level(a, b)
        qs = self.qs(a.level)
        d0 = C.mul(a.data[0], b.data[0], qs)
        d1 = C.add(C.mul(a.data[0], b.data[1], qs), C.mul(a.data[1], b.data[0], qs), qs)
        d2 = C.mul(a.data[1], b.data[1], qs)
        return np.stack([d0, d1, d2]), a.scale * b.scale

    def _check_level(self, a, b):
        if a.level != b.level:
            raise ValueError("level mismatch")

    def relin(self, d, scale, key):
        """Key-switch d2 from s^2 to s: (d0 + u0, d1 + u1)."""
        level = d.shape[1]
        qs = self.qs(level)
        ext = self.modup(d[2], level)
        u0, u1 = self.keyswitch_ext(ext, key, 1, level)
        return Ciphertext(np.stack([C.add(d[0], u0, qs), C.add(d[1], u1, qs)]), scale)

    def mul_relin(self, a, b, key):
        d, s = self.tensor(a, b)
        return self.relin(d, s, key)
