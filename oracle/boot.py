"""CKKS bootstrapping oracle -- TEST INFRASTRUCTURE ONLY.

The paper refreshes a ciphertext's levels with its CPU library's CKKS
bootstrapping: a support function the user places between layers (section
"FHEON's Support Functions"), and the deep models of the evaluation section
bootstrap before most activations.  The paper does not describe the
procedure, so this module writes out the standard four-stage RNS-CKKS
bootstrapping with every open choice pinned, composed only of the oracle's
exact ring operations (``ckks.Context``) and its Chebyshev evaluation
(``layers.cheb_eval``), so that a GPU composition of the same steps can be
held to it bit for bit:

1. ModRaise (``mod_raise``): the level-1 ciphertext's residues mod q_0, read
   centred in (-q_0/2, q_0/2], reduced modulo every prime of the chain.  It
   now encrypts t = m + q_0 I for a small integer polynomial I.
2. CoeffToSlot (``linear_transform`` over ``cts_groups``): the inverse of the
   slot decoding map as a product of radix-2 butterfly factors (the special
   FFT of the power-of-5 root order, ``stage_diags``), grouped into a few
   levels, each level evaluated by baby-step giant-step diagonals.  Its
   output holds (t_lo + i t_hi) / (2 q_0 K) in bit-reversed slot order.
3. EvalMod: conjugation splits real and imaginary parts; each goes through
   the Chebyshev interpolant of sin(2 pi K x) / (2 pi) (``mod_coeffs``), or
   of cos(2 pi (K x - 1/4) / 2^r) followed by r double angles
   c <- 2 c^2 - 1 (which end at sin(2 pi K x)) and a scale label times
   2 pi; either way q_0 I is removed and about m / q_0 remains.
4. SlotToCoeff: the forward butterfly factors, bit-reversed input to natural
   order, give back the slot vector of m.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It imports nothing from the GPU package.

Parity status: ModRaise is pinned by exact integer identities (tests/
test_oracle_boot.py: residues against Python big integers, t = m + q_0 I
with |I| within the secret's bound); the butterfly factors against direct
evaluation of the decoding sums and against the oracle's FFT decoder; the
baby-step giant-step evaluation against dense matrix-vector products in a
plain complex slot simulation; the EvalMod coefficients against the sine on
a dense grid; the whole procedure by decryption (the refreshed ciphertext
decrypts to the input's message within the bound derived there).
"""
import math

import numpy as np

from . import _lib as C
from . import layers as LY
from .ckks import CONJ, Ciphertext, Plaintext


# ===================================================================== ModRaise
def mod_raise(ctx, ct, level):
    """Residues of c0, c1 mod q_0 (limb 0, NTT form) -> the same integers,
    read centred, modulo q_0..q_{level-1} (NTT form).  Coefficient a in
    [0, q_0) is read as a if a <= (q_0 - 1) / 2, else a - q_0.  The scale is
    unchanged; limb 0 of the result equals limb 0 of the input."""
    q0 = ctx.pr.q[0]
    qs, ps = ctx.qs(level), ctx.psis(level)
    out = np.empty((2, level, ctx.n), dtype=np.uint64)
    for k in range(2):
        a = ctx.intt(ct.data[k, :1], [q0], [ctx.pr.psi[0]])[0]
        signed = np.where(a > q0 // 2, a.astype(np.int64) - np.int64(q0), a.astype(np.int64))
        out[k] = ctx.ntt(C.from_signed(signed, qs), qs, ps)
    return Ciphertext(out, ct.scale)


def monomial_pt(ctx, e, level):
    """The plaintext X^e (e in [0, 2N)), NTT form over q_0..q_{level-1},
    scale 1.  Multiplying by X^(N/2) multiplies every slot by i (the slot
    roots are zeta^(5^j) and 5^j = 1 mod 4), by X^(3N/2) = -X^(N/2) by -i."""
    n = ctx.n
    poly = np.zeros(n, dtype=np.int64)
    poly[e % n] = 1 if (e // n) % 2 == 0 else -1
    qs = ctx.qs(level)
    return Plaintext(ctx.ntt(C.from_signed(poly, qs), qs, ctx.psis(level)), 1.0)


# ===================================================================== special FFT factors
def slot_root(m, j):
    """x_{m,j} = exp(2 pi i 5^j / (4m)): the point where a size-m
    sub-problem of the decoding map evaluates its j-th output (m a power of
    two, the full map m = N/2 at zeta^(5^j), zeta = exp(i pi / N))."""
    return np.exp(2j * np.pi * pow(5, j, 4 * m) / (4 * m))


def _put(d, shift, vec):
    if shift in d:
        d[shift] = d[shift] + vec
    else:
        d[shift] = vec


def stage_diags(n, h, inverse):
    """One radix-2 butterfly stage of block size 2h on an n-slot vector, as
    diagonals {shift: vector} (y[p] = sum_d D_d[p] x[(p + d) mod n]).
    Forward (decimation in time, bit-reversed input): for p = s + j in the
    first half of its block (j < h) y[p] = x[p] + x_{2h,j} x[p + h], and for
    p = s + j + h y[p] = x[p - h] - x_{2h,j} x[p].  The inverse stage is
    x[p] = (y[p] + y[p + h]) / 2, x[p + h] = (y[p] - y[p + h]) / (2 x_{2h,j}).
    (x_{2h, j+h} = -x_{2h, j} because 5^h = 1 + 4h mod 8h.)"""
    p = np.arange(n)
    r = p % (2 * h)
    first = r < h
    roots = np.array([slot_root(2 * h, j) for j in range(h)])
    x = roots[np.where(first, r, r - h)]
    if inverse:
        d0 = np.where(first, 0.5 + 0j, -0.5 / x)
        dp = np.where(first, 0.5 + 0j, 0j)
        dm = np.where(first, 0j, 0.5 / x)
    else:
        d0 = np.where(first, 1.0 + 0j, -x)
        dp = np.where(first, x, 0j)
        dm = np.where(first, 0j, 1.0 + 0j)
    out = {0: d0}
    _put(out, h % n, dp)
    _put(out, (-h) % n, dm)
    return out


def compose(a, b, n):
    """Diagonals of the product A B (B applied first):
    C_{(d+e) mod n}[p] += A_d[p] B_e[(p + d) mod n].  Diagonals that are
    identically zero are dropped."""
    out = {}
    for d in sorted(a):
        for e in sorted(b):
            _put(out, (d + e) % n, a[d] * np.roll(b[e], -d))
    return {k: v for k, v in out.items() if np.any(v != 0)}


def group_sizes(log_slots, levels):
    """Stages per level: as even as possible, the larger groups first."""
    q, r = divmod(log_slots, levels)
    return [q + 1] * r + [q] * (levels - r)


def cts_groups(log_slots, levels):
    """CoeffToSlot's inverse stages in application order (block half-size h
    from N/4 down to 1), split into `levels` groups."""
    hs = [1 << s for s in range(log_slots - 1, -1, -1)]
    out, at = [], 0
    for g in group_sizes(log_slots, levels):
        out.append(hs[at:at + g])
        at += g
    return out


def stc_groups(log_slots, levels):
    """SlotToCoeff's forward stages in application order (h from 1 up):
    CoeffToSlot's groups mirrored."""
    return [list(reversed(g)) for g in reversed(cts_groups(log_slots, levels))]


def group_diags(n, hs, inverse):
    """Diagonals of one level: the product of its stages, the first of `hs`
    applied first."""
    m = {0: np.ones(n, dtype=np.complex128)}
    for h in hs:
        m = compose(stage_diags(n, h, inverse), m, n)
    return m


# ===================================================================== baby-step giant-step
def centred(k, m):
    """k mod m in (-m/2, m/2]."""
    k %= m
    return k - m if k > m // 2 else k


class LevelPlan:
    """Baby-step giant-step layout of one level's diagonals.  Every shift is
    a multiple of the level's smallest stage u; shift d is written
    u k, k = d / u centred modulo n / u, and k = i + B j with
    B = the smallest power of two with B^2 >= kmax - kmin + 1, baby step
    i in [0, B), giant step j (floor division).  `giants` lists, for every j
    in ascending order with a term, its (i, shift) pairs in ascending i;
    `babies` the baby steps i > 0 used."""

    def __init__(self, shifts, n, u):
        self.n, self.u = n, u
        m = n // u
        ks = sorted(centred(d // u, m) for d in shifts)
        span = ks[-1] - ks[0] + 1
        B = 1
        while B * B < span:
            B *= 2
        self.B = B
        by_j = {}
        for k in ks:
            j, i = k // B, k % B
            by_j.setdefault(j, []).append((i, (u * k) % n))
        self.giants = [(j, sorted(by_j[j])) for j in sorted(by_j)]
        self.babies = sorted({i for _, t in self.giants for i, _ in t if i > 0})

    def baby_rot(self, i):
        return (self.u * i) % self.n

    def giant_rot(self, j):
        return (self.u * self.B * j) % self.n

    def rotations(self):
        """Rotation amounts (mod n) the level uses: baby steps, then giant steps."""
        rots = {self.baby_rot(i) for i in self.babies}
        rots |= {self.giant_rot(j) for j, _ in self.giants if j != 0}
        return rots - {0}

    def count(self):
        return sum(len(t) for _, t in self.giants)


def level_plaintext_values(diags, plan):
    """The level's plaintext vectors in consumption order (giant j
    ascending, baby i ascending): diagonal D_d pre-rotated by the giant
    step, rot(D_d, -u B j)[p] = D_d[p - u B j]."""
    out = []
    for j, terms in plan.giants:
        for _, d in terms:
            out.append(np.roll(diags[d], plan.u * plan.B * j))
    return out


def linear_transform(ev, x, plan, pts):
    """y = sum_d D_d (.) Rot_d(x) by baby-step giant-step:
    babies r_i = Rot_{u i}(x) (one hoisted set; r_0 = x);
    for every giant j (ascending): s_j = RS(sum_i pt_{j,i} (.) r_i), then
    Rot_{u B j}(s_j) unless j = 0 (rescaled before its key switch); y is the
    sum of these.  pts in consumption order (``level_plaintext_values``)."""
    rots = [plan.baby_rot(i) for i in plan.babies]
    baby = dict(zip(plan.babies, ev.rot_hoisted(x, rots))) if rots else {}
    baby[0] = x
    acc, t = None, 0
    for j, terms in plan.giants:
        s = LY.mac(ev, [baby[i] for i, _ in terms], pts[t:t + len(terms)])
        t += len(terms)
        s = ev.rescale(s)
        if j != 0:
            s = ev.rot(s, plan.giant_rot(j))
        acc = s if acc is None else ev.add(acc, s)
    return acc


# ===================================================================== plan of the whole procedure
class BootPlan:
    """Everything the procedure needs besides keys and ciphertexts, for
    N/2 = n slots, `levels` levels per linear transform, a bound k_min on
    |I| + 1/2 (I the multiple of q_0 that ModRaise adds), base scale delta
    (the EvalMod input's scale), a Chebyshev degree and a number r of
    double angles (0: the sine is interpolated directly).

    The raised ciphertext is relabelled 2^e delta with e the smallest
    integer such that 2^e delta >= 2 q_0 k_min, and EvalMod's range is
    K = 2^e delta / (2 q_0) (>= k_min): CoeffToSlot then lands
    t / (2 q_0 K) and its plaintext scales (q 2^-e_g, the e_g summing to e)
    bring the scale back to delta up to the primes' ratios q / q, which the
    Chebyshev evaluation needs (its squarings double any gap between the
    input scale and the primes)."""

    def __init__(self, log_n, levels, k_min, delta, degree, double_angles=0):
        self.log_n, self.levels, self.k_min, self.delta, self.degree = log_n, levels, k_min, delta, degree
        self.double_angles = double_angles
        self.n = 1 << (log_n - 1)
        ls = log_n - 1
        self.cts_hs = cts_groups(ls, levels)
        self.stc_hs = stc_groups(ls, levels)
        self.cts_diags = [group_diags(self.n, hs, True) for hs in self.cts_hs]
        self.stc_diags = [group_diags(self.n, hs, False) for hs in self.stc_hs]
        self.cts_plans = [LevelPlan(sorted(d), self.n, min(hs)) for d, hs in zip(self.cts_diags, self.cts_hs)]
        self.stc_plans = [LevelPlan(sorted(d), self.n, min(hs)) for d, hs in zip(self.stc_diags, self.stc_hs)]

    def rotations(self):
        """Rotation amounts (mod N/2) of both transforms, ascending; the
        conjugation key comes on top."""
        r = set()
        for p in self.cts_plans + self.stc_plans:
            r |= p.rotations()
        return sorted(r)

    def cts_values(self):
        return [level_plaintext_values(d, p) for d, p in zip(self.cts_diags, self.cts_plans)]

    def stc_values(self):
        return [level_plaintext_values(d, p) for d, p in zip(self.stc_diags, self.stc_plans)]

    def raise_exp(self, q0):
        e, bound = 0, 2.0 * float(q0) * self.k_min
        while math.ldexp(self.delta, e) < bound:
            e += 1
        return e

    def raise_scale(self, q0):
        return math.ldexp(self.delta, self.raise_exp(q0))

    def K(self, q0):
        return self.raise_scale(q0) / (2.0 * float(q0))

    def cts_exponents(self, q0):
        """e_g of CoeffToSlot level g's plaintext scale q 2^-e_g: e split as
        evenly as possible, larger first."""
        return group_sizes(self.raise_exp(q0), self.levels)

    def stc_exponents(self, q0):
        """f_g of SlotToCoeff level g's plaintext scale q 2^f_g: f =
        round(log2(q_0 / (delta a))) (a = 2 pi with double angles, else 1:
        EvalMod's output label) split as evenly as possible, so that the
        result's scale label comes back near the input's (EvalMod returns
        m / q_0 at scale delta a)."""
        a = 2.0 * math.pi if self.double_angles else 1.0
        f = int(math.floor(math.log2(float(q0) / (self.delta * a)) + 0.5))
        return group_sizes(f, self.levels) if f > 0 else [0] * self.levels

    def mod_coeffs(self, q0):
        return mod_coeffs(self.K(q0), self.degree, self.double_angles)

    def evalmod_levels(self, q0):
        return LY.cheb_plan(self.mod_coeffs(q0), False)[0] + self.double_angles


def mod_coeffs(K, degree, double_angles=0):
    """Chebyshev interpolant on [-1, 1] at the degree + 1 first-kind nodes
    x_k = cos(pi (k + 1/2) / (degree + 1)): c_j = 2 / (degree + 1)
    sum_k f(x_k) T_j(x_k), f ~ c_0 / 2 + sum c_j T_j, of
      r = 0: f(x) = sin(2 pi K x) / (2 pi) (odd: even coefficients set to 0);
      r > 0: f(x) = cos(2 pi (K x - 1/4) / 2^r), whose r double angles give
             cos(2 pi K x - pi / 2) = sin(2 pi K x).
    For x = t / (q_0 K), t = m + q_0 I: sin(2 pi K x) = sin(2 pi m / q_0),
    about 2 pi m / q_0."""
    n = degree + 1
    theta = np.pi * (np.arange(n) + 0.5) / n
    if double_angles:
        fx = np.cos(2.0 * np.pi * (K * np.cos(theta) - 0.25) / float(1 << double_angles))
    else:
        fx = np.sin(2.0 * np.pi * K * np.cos(theta)) / (2.0 * np.pi)
    c = np.array([2.0 / n * float(np.sum(fx * np.cos(j * theta))) for j in range(n)])
    if not double_angles:
        c[0::2] = 0.0
    return c


def evalmod(ev, x, plan, coeffs):
    """One EvalMod part: c = cheb_eval(x, coeffs, no mask, delta); then r
    times p = RS(Relin(c c)), c = (p + p) - 1; with r > 0 the scale label is
    multiplied by 2 pi (c then decodes to about m / q_0)."""
    c = LY.cheb_eval(ev, x, coeffs, None, plan.delta)
    for _ in range(plan.double_angles):
        p = ev.rescale(ev.mul_relin(c, c))
        c = ev.add_const(ev.add(p, p), -1.0)
    if plan.double_angles:
        c = Ciphertext(c.data, c.scale * (2.0 * math.pi))
    return c


def encode_level(ctx, values, scale, level):
    """Complex slot vectors -> NTT-form plaintexts at `level` and `scale`."""
    return [ctx.encode_complex(v, scale, level) for v in values]


def boot_plaintexts(ctx, plan, level_in):
    """Encoded CoeffToSlot and SlotToCoeff plaintexts for a raise to
    `level_in`: CoeffToSlot level g at level_in - g with scale
    q_{level_in-g-1} 2^-e_g; SlotToCoeff level g at its own level l with
    scale q_{l-1} 2^f_g."""
    q = ctx.pr.q
    cts, stc = [], []
    ex = plan.cts_exponents(q[0])
    for g, vals in enumerate(plan.cts_values()):
        lv = level_in - g
        cts.append(encode_level(ctx, vals, math.ldexp(float(q[lv - 1]), -ex[g]), lv))
    lv0 = level_in - plan.levels - plan.evalmod_levels(q[0])
    fx = plan.stc_exponents(q[0])
    for g, vals in enumerate(plan.stc_values()):
        lv = lv0 - g
        stc.append(encode_level(ctx, vals, math.ldexp(float(q[lv - 1]), fx[g]), lv))
    return cts, stc


def bootstrap(ctx, ct, plan, keys, relin_key, cts_pts, stc_pts, level_in=None):
    """The refreshed ciphertext of `ct` (any level; limb 0 is used):
      x  = ModRaise(ct) to level_in (default L), relabelled 2^e delta = 2 q_0 K;
      CoeffToSlot: x = linear_transform(level g) for g = 0..levels-1;
      w  = Rot_conj(x);  re = x + w;  im = (-X^(N/2)) (.) (x - w);
      re, im = evalmod(.) (Chebyshev series, r double angles);
      z  = re + X^(N/2) (.) im;
      SlotToCoeff: z = linear_transform(level g) for g = 0..levels-1;
      result = z relabelled scale(z) * scale(ct) / q_0 (z's slots hold the
      message times scale(ct) / q_0).
    Levels consumed: 2 levels + cheb levels + r; key switches: the
    transforms' rotations, one conjugation, the Chebyshev and double-angle
    relinearizations (twice)."""
    L = level_in or ctx.pr.L
    ev = LY.HEEval(ctx, keys, relin_key)
    x = mod_raise(ctx, ctx.drop_level(ct, 1), L)
    x = Ciphertext(x.data, plan.raise_scale(ctx.pr.q[0]))
    for p, pts in zip(plan.cts_plans, cts_pts):
        x = linear_transform(ev, x, p, pts)
    w = ev.rot(x, CONJ)
    re = ctx.add(x, w)
    im = ctx.mul_plain(ctx.sub(x, w), monomial_pt(ctx, 3 * ctx.n // 2, x.level))
    coeffs = plan.mod_coeffs(ctx.pr.q[0])
    re = evalmod(ev, re, plan, coeffs)
    im = evalmod(ev, im, plan, coeffs)
    z = ctx.add(re, ctx.mul_plain(im, monomial_pt(ctx, ctx.n // 2, im.level)))
    for p, pts in zip(plan.stc_plans, stc_pts):
        z = linear_transform(ev, z, p, pts)
    return Ciphertext(z.data, z.scale * (ct.scale / float(ctx.pr.q[0]))), ev.ks
