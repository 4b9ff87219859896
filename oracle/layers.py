"""FHEON's secure CNN layers as pinned CKKS schedules — TEST INFRASTRUCTURE ONLY.

Written from the paper's section "Secure Neural Network Layers":
  * feature maps are flattened channel by channel into one SIMD vector
    (Fig. "Flattening of an input tensor"); slot c*cs + y*rs + x = X[c, y, x];
  * a convolution rotates the input to align every kernel tap, multiplies each
    rotated copy by a vector of the repeated kernel value and sums
    (Secure Convolution Layer); input channels are summed by repeated
    rotations with the single key W^2; out-channels are placed by rotations
    by multiples of the channel block;
  * the 3x3 / stride 1 / pad 1 case uses the rotation tree of Algorithm 1
    and the nine masks of Algorithms 2-3 instead of explicit padding
    (Special Secure Convolution Layer);
  * striding extracts the stride-aligned outputs with masks and rotations,
    jointly for all channels (Secure Advanced Convolution With Striding,
    approach 1, or approach 2's log-step column moves, and the
    multi-channel pipeline);
  * padding beyond (k-1)/2 re-lays the input out as the padded tensor
    (Secure Advanced Convolution With Padding);
  * average pooling sums the window rotations and multiplies by 1/k^2, then
    strides; global average pooling sums each W^2 block and merges the
    channels; the fully connected layer multiplies by each weight row, sums
    n slots and consolidates the m outputs with rotations;
  * the secure ReLU (section "Activation Function (Secure ReLU)" and its
    algorithm) scales the input by 1/beta with a mask when beta > 1 and
    evaluates the degree-D Chebyshev interpolant of f(z) = beta max(0, z)
    on [-1, 1] (D = 59 by default).
The exact rotation amounts, mask contents and rescale placement are this
project's pinned reading (the paper leaves them open); the GPU library
implements the same schedule independently.

Each schedule is written once against an evaluator: ``HEEval`` runs it with
the oracle's CKKS arithmetic, ``SimEval`` with plain float64 slot vectors
(np.roll for rotations) so that the schedule itself can be pinned against the
paper's FP64 layer equations.
"""
import math

import numpy as np

# degree-4 least-squares fit of max(0, x) on [-1, 1] (uniform weight):
# projection of |x| on Legendre P0, P2, P4 gives 15/128 + 105/64 x^2 - 105/128 x^4,
# and max(0, x) = (|x| + x) / 2.
RELU4 = {0: 15.0 / 256.0, 1: 0.5, 2: 105.0 / 128.0, 4: -105.0 / 256.0}


CHEB_DEGREE = 59  # the paper's default Chebyshev degree for the secure ReLU


# ===================================================================== FP64 references
def conv2d_ref(X, K, stride=1, padding=0, bias=None):
    """Y[f, h, w] = sum_{c,i,j} X[c, S h + i - P, S w + j - P] K[f, c, i, j] + b_f
    (zero outside the input), output size (H + 2P - k)/S + 1."""
    C, H, W = X.shape
    F, C2, kh, kw = K.shape
    assert C == C2
    Ho = (H + 2 * padding - kh) // stride + 1
    Wo = (W + 2 * padding - kw) // stride + 1
    Y = np.zeros((F, Ho, Wo))
    for f in range(F):
        for h in range(Ho):
            for w in range(Wo):
                acc = 0.0
                for c in range(C):
                    for i in range(kh):
                        for j in range(kw):
                            y, x = stride * h + i - padding, stride * w + j - padding
                            if 0 <= y < H and 0 <= x < W:
                                acc += X[c, y, x] * K[f, c, i, j]
                Y[f, h, w] = acc + (bias[f] if bias is not None else 0.0)
    return Y


def avgpool_ref(X, k, stride):
    """Output(i, j) = (1/k^2) sum_{x,y < k} Input(S i + x, S j + y) per channel."""
    C, H, W = X.shape
    Ho, Wo = (H - k) // stride + 1, (W - k) // stride + 1
    Y = np.zeros((C, Ho, Wo))
    for c in range(C):
        for i in range(Ho):
            for j in range(Wo):
                Y[c, i, j] = X[c, stride * i:stride * i + k, stride * j:stride * j + k].sum() / (k * k)
    return Y


def gap_ref(X):
    return X.reshape(X.shape[0], -1).mean(axis=1)


def fc_ref(x, Wm, b=None):
    """y_k = sum_i W_ki x_i + b_k."""
    y = np.array([sum(Wm[k, i] * x[i] for i in range(len(x))) for k in range(Wm.shape[0])])
    return y if b is None else y + b


def relu4_ref(x):
    return RELU4[0] + RELU4[1] * x + RELU4[2] * x ** 2 + RELU4[4] * x ** 4


# ===================================================================== masks (Alg. 2 / 3)
def neighbour_masks(W):
    """Closed form: tap (dy, dx) of output pixel (y, x) reads inside the image."""
    out = []
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            m = np.zeros(W * W)
            for y in range(W):
                for x in range(W):
                    if 0 <= y + dy < W and 0 <= x + dx < W:
                        m[y * W + x] = 1.0
            out.append(m)
    return out


def special_masks(W, C):
    """The nine 0/1 masks of the 3x3 / stride 1 / pad 1 convolution (what
    Algorithms 2 and 3 of the special convolution produce: zeros where a
    tap would read across the image border), tap k = 3 (dy + 1) + (dx + 1),
    one W^2 block per input channel.  Built from the closed form of
    ``neighbour_masks``, repeated over the C channels."""
    return [np.tile(m, C) for m in neighbour_masks(W)]


# ===================================================================== geometry
class FMap:
    """Feature-map layout in the slots: channel c, row y, column x at
    c*cs + y*rs + x for c < C, y < H, x < W; reps = 2 when the C-channel
    block is stored twice back to back."""

    def __init__(self, C, H, W, rs=None, cs=None, reps=1):
        self.C, self.H, self.W = C, H, W
        self.rs = W if rs is None else rs
        self.cs = H * self.rs if cs is None else cs
        self.reps = reps

    def key(self):
        return (self.C, self.H, self.W, self.rs, self.cs, self.reps)

    def __eq__(self, o):
        return self.key() == o.key()

    def __repr__(self):
        return "FMap(C=%d,H=%d,W=%d,rs=%d,cs=%d,reps=%d)" % self.key()


def pack(X, fm, slots):
    """Real slot vector holding tensor X (C,H,W) in layout fm."""
    v = np.zeros(slots)
    for r in range(fm.reps):
        for c in range(fm.C):
            for y in range(fm.H):
                base = (r * fm.C + c) * fm.cs + y * fm.rs
                v[base:base + fm.W] = X[c, y]
    return v


def unpack(v, fm):
    X = np.zeros((fm.C, fm.H, fm.W))
    for c in range(fm.C):
        for y in range(fm.H):
            base = c * fm.cs + y * fm.rs
            X[c, y] = v[base:base + fm.W]
    return X


# ===================================================================== evaluators
class SimCt:
    def __init__(self, v, level, scale=1.0):
        self.v, self.level, self.scale = v, level, scale


class SimEval:
    """Plain float64 slot simulation of a schedule (no encryption)."""

    def __init__(self, slots):
        self.slots = slots
        self.ks = 0

    def rot_hoisted(self, x, rs):
        self.ks += sum(1 for r in rs if r % self.slots)
        return [SimCt(np.roll(x.v, -r), x.level, x.scale) for r in rs]

    def rot(self, x, r):
        return self.rot_hoisted(x, [r])[0]

    def mul_plain(self, x, pt):
        return SimCt(x.v * pt, x.level, x.scale)

    def add(self, a, b):
        assert a.level == b.level
        return SimCt(a.v + b.v, a.level, a.scale)

    def rescale(self, x):
        return SimCt(x.v, x.level - 1, x.scale)

    def drop(self, x, level):
        return SimCt(x.v, level, x.scale)

    def mul_relin(self, a, b):
        assert a.level == b.level
        return SimCt(a.v * b.v, a.level, a.scale)

    def add_plain(self, x, pt):
        return SimCt(x.v + pt, x.level, x.scale)

    def mul_const(self, x, c, scale):
        return SimCt(x.v * c, x.level, x.scale)

    def add_const(self, x, c):
        return SimCt(x.v + c, x.level, x.scale)

    def with_scale(self, x, s):
        return SimCt(x.v, x.level, s)

    def modulus(self, level_index):
        return 2.0 ** 40


class HEEval:
    """The same schedule with the oracle's CKKS arithmetic."""

    def __init__(self, ctx, keys, relin_key=None):
        self.ctx, self.keys, self.relin_key = ctx, keys, relin_key
        self.ks = 0

    def rot_hoisted(self, x, rs):
        self.ks += sum(1 for r in rs if self.ctx.galois_element(r) != 1)
        return self.ctx.rotate_hoisted(x, rs, self.keys)

    def rot(self, x, r):
        return self.rot_hoisted(x, [r])[0]

    def mul_plain(self, x, pt):
        return self.ctx.mul_plain(x, pt)

    def add(self, a, b):
        return self.ctx.add(a, b)

    def rescale(self, x):
        return self.ctx.rescale(x)

    def drop(self, x, level):
        return self.ctx.drop_level(x, level)

    def mul_relin(self, a, b):
        self.ks += 1
        return self.ctx.mul_relin(a, b, self.relin_key)

    def add_plain(self, x, pt):
        return self.ctx.add_plain(x, pt)

    def mul_const(self, x, c, scale):
        return self.ctx.mul_plain(x, self.ctx.encode_const(c, scale, x.level))

    def add_const(self, x, c):
        return self.ctx.add_plain(x, self.ctx.encode_const(c, x.scale, x.level))

    def with_scale(self, x, s):
        from .ckks import Ciphertext

        return Ciphertext(x.data, s)

    def modulus(self, level_index):
        return self.ctx.pr.q[level_index]


# ===================================================================== schedule pieces
def mac(ev, cts, pts):
    """sum_t ct_t (.) pt_t (one multiplicative level, not rescaled)."""
    acc = None
    for c, p in zip(cts, pts):
        t = ev.mul_plain(c, p)
        acc = t if acc is None else ev.add(acc, t)
    return acc


def horner(ev, terms_fn, n, key):
    """sum_{t<n} Rot_{t*key}(RS(term_t)) evaluated as
    acc = RS(term_{n-1}); acc = Rot_key(acc) + RS(term_t) for t = n-2..0."""
    acc = ev.rescale(terms_fn(n - 1))
    for t in range(n - 2, -1, -1):
        acc = ev.add(ev.rot(acc, key), ev.rescale(terms_fn(t)))
    return acc


def bsgs_split(n):
    """Baby steps B = ceil(sqrt(n)) and giant steps A = ceil(n / B) of a masked chain."""
    B = math.isqrt(n - 1) + 1 if n > 1 else 1
    return B, (n + B - 1) // B


def masked_chain_keys(n, key, bsgs):
    """Rotation keys of masked_chain."""
    if n <= 1:
        return set()
    if not bsgs:
        return {key}
    B, A = bsgs_split(n)
    return {b * key for b in range(1, B)} | ({B * key} if A > 1 else set())


def masked_chain_switches(n, bsgs):
    if n <= 1:
        return 0
    if not bsgs:
        return n - 1
    B, A = bsgs_split(n)
    return (B - 1) + (A - 1)


def chain_masks(vecs, key, bsgs):
    """Mask vectors of a masked chain: as given (Horner), or for the baby-step
    giant-step chain mask t = a B + b pre-rotated by b key (Rot_r moves slot
    i + r to slot i, i.e. np.roll by -r)."""
    if not bsgs:
        return list(vecs)
    B, _ = bsgs_split(len(vecs))
    return [np.roll(m, -(t % B) * key) for t, m in enumerate(vecs)]


def masked_chain(ev, v, masks, n, key, bsgs=False):
    """sum_{t<n} Rot_{t key}(v (.) m_t), one level.

    Horner (default): acc = RS(v.m_{n-1}); acc = Rot_key(acc) + RS(v.m_t),
    n - 1 key switches.  Baby-step giant-step: with t = a B + b,
    Rot_{t key}(v.m_t) = Rot_{a B key}(Rot_{b key}(v) . Rot_{b key}(m_t)), so
    with the pre-rotated masks m'_t (chain_masks) the inner sums
    I_a = RS(sum_b Rot_{b key}(v) . m'_{aB+b}) use one hoisted group of B - 1
    rotations of v, and acc = I_{A-1}; acc = Rot_{B key}(acc) + I_a adds
    A - 1 more.
    """
    if not bsgs:
        return horner(ev, lambda t: ev.mul_plain(v, masks[t]), n, key)
    B, A = bsgs_split(n)
    baby = [v] + (ev.rot_hoisted(v, [b * key for b in range(1, B)]) if B > 1 else [])

    def inner(a):
        idx = [t for t in range(a * B, min(n, a * B + B))]
        return ev.rescale(mac(ev, [baby[t - a * B] for t in idx], [masks[t] for t in idx]))

    acc = inner(A - 1)
    for a in range(A - 2, -1, -1):
        acc = ev.add(ev.rot(acc, B * key), inner(a))
    return acc


def log_steps(Wo):
    """ceil(log2 Wo): the column steps of the log-step extraction."""
    return (Wo - 1).bit_length()


def compaction_plan(fm, S, Ho, Wo, stride_log=False, multi=None):
    """Steps of the stride-S extraction of outputs (S i, S j), jointly over all
    channels: (i) columns, key S-1 (the paper's first striding approach: one
    masked chain over the Wo columns), or with stride_log (its second
    approach) ceil(log2 Wo) steps t with key (S-1) 2^t, each a two-term
    masked chain keeping the columns whose bit t is 0 and moving those whose
    bit t is 1 left by (S-1) 2^t; (ii) rows, key D = S rs - Wo;
    (iii) channels, key E = cs - Ho Wo, when there are several channels
    (multi; a one-channel group of the multi-channel pipeline keeps the step
    as one mask, so that every group ends at the same level).  Returns
    [(step, count, key)]."""
    steps = []
    if S > 1:
        T = log_steps(Wo)
        if stride_log and T > 0:
            steps += [("logcol%d" % t, 2, (S - 1) << t) for t in range(T)]
        else:
            steps.append(("col", Wo, S - 1))
    D = S * fm.rs - Wo
    if D != 0:
        steps.append(("row", Ho, D))
    E = fm.cs - Ho * Wo
    if E != 0 and (fm.C > 1 if multi is None else multi):
        steps.append(("chan", fm.C, E))
    return steps


def compaction_masks(fm, S, Ho, Wo, col_scale, slots, bsgs=False, stride_log=False, c0=0, multi=None):
    """Masks of each step on the layout that step sees.  Log-step column step
    t: after steps < t, column j of the stride-S row i sits at
    S i rs + S (j - j mod 2^t) + j mod 2^t; mask 0 is 1 there for the j with
    bit t clear (they stay), mask 1 for those with bit t set (they move by
    (S-1) 2^t); step 0 also selects the stride-aligned outputs, and carries
    the column scale.  c0: the channels are c0 .. c0 + C - 1 of the map (a
    group of the multi-channel pipeline, see strided)."""
    vecs = []
    for step, n, key in compaction_plan(fm, S, Ho, Wo, stride_log, multi):
        sv = []
        for t in range(n):
            m = np.zeros(slots)
            for c in range(c0, c0 + fm.C):
                if step.startswith("logcol"):
                    lt = int(step[6:])
                    for i in range(Ho):
                        for j in range(Wo):
                            if (j >> lt) & 1 == t:
                                b = j & ((1 << lt) - 1)
                                pos = S * (j - b) + b
                                m[c * fm.cs + S * i * fm.rs + pos] = col_scale if lt == 0 else 1.0
                elif step == "col":
                    for i in range(Ho):
                        m[c * fm.cs + S * i * fm.rs + S * t] = col_scale
                elif step == "row":
                    base = c * fm.cs + S * t * fm.rs
                    m[base:base + Wo] = 1.0
                elif step == "chan" and c == c0 + t:
                    m[c * fm.cs:c * fm.cs + Ho * Wo] = 1.0
            sv.append(m)
        vecs += chain_masks(sv, key, bsgs)
    return vecs


def compaction_keys(fm, S, Ho, Wo, bsgs=False, stride_log=False, multi=None):
    keys = set()
    for _, n, key in compaction_plan(fm, S, Ho, Wo, stride_log, multi):
        keys |= masked_chain_keys(n, key, bsgs)
    return keys


def compaction(ev, v, fm, S, Ho, Wo, masks, bsgs=False, stride_log=False, multi=None):
    """Move output (c, i, j) from c cs + S i rs + S j to c Ho Wo + i Wo + j
    (channels offset by c0 of a group keep c0 cs as their origin:
    c0 cs + c Ho Wo + i Wo + j, see strided)."""
    pos = 0
    for step, n, key in compaction_plan(fm, S, Ho, Wo, stride_log, multi):
        ms = masks[pos:pos + n]
        pos += n
        v = masked_chain(ev, v, ms, n, key, bsgs)
    assert pos == len(masks)
    return v, FMap(fm.C, Ho, Wo, Wo, Ho * Wo, 1)


def stride_groups(C, g):
    """The multi-channel striding pipeline's groups [(c0, size)]: g output
    channels each (the paper sets g to the layer's input channels); g <= 0 or
    g >= C is one group of all C channels."""
    if g <= 0 or g >= C:
        return [(0, C)]
    return [(c0, min(g, C - c0)) for c0 in range(0, C, g)]


def strided_masks(fm, S, Ho, Wo, col_scale, slots, bsgs=False, stride_log=False, group=0):
    """compaction_masks of every group in turn (the merge takes none)."""
    out = []
    for c0, n in stride_groups(fm.C, group):
        out += compaction_masks(FMap(n, fm.H, fm.W, fm.rs, fm.cs, 1), S, Ho, Wo, col_scale, slots, bsgs, stride_log,
                                c0, fm.C > 1)
    return out


def strided_keys(fm, S, Ho, Wo, bsgs=False, stride_log=False, group=0):
    groups = stride_groups(fm.C, group)
    keys = set()
    for _, n in groups:
        keys |= compaction_keys(FMap(n, fm.H, fm.W, fm.rs, fm.cs, 1), S, Ho, Wo, bsgs, stride_log, fm.C > 1)
    if len(groups) > 1:
        keys.add(group * (fm.cs - Ho * Wo))
    return keys


def strided(ev, v, fm, S, Ho, Wo, masks, bsgs=False, stride_log=False, group=0):
    """Stride compaction of all channels (group 0) or, the paper's
    multi-channel pipeline, of groups of `group` channels each: group c0's
    compaction leaves its channel c at c0 cs + c Ho Wo, i.e. c0 E = c0 (cs -
    Ho Wo) to the right of its place, so the groups are merged by a Horner
    chain with the single key group E: acc = z_last; acc = Rot_{gE}(acc) +
    z_k (no level)."""
    groups = stride_groups(fm.C, group)
    zs, pos = [], 0
    for c0, n in groups:
        sub = FMap(n, fm.H, fm.W, fm.rs, fm.cs, 1)
        cnt = sum(k for _, k, _ in compaction_plan(sub, S, Ho, Wo, stride_log, fm.C > 1))
        z, _ = compaction(ev, v, sub, S, Ho, Wo, masks[pos:pos + cnt], bsgs, stride_log, fm.C > 1)
        zs.append(z)
        pos += cnt
    assert pos == len(masks)
    acc = zs[-1]
    for z in reversed(zs[:-1]):
        acc = ev.add(ev.rot(acc, group * (fm.cs - Ho * Wo)), z)
    return acc, FMap(fm.C, Ho, Wo, Wo, Ho * Wo, 1)


# ===================================================================== convolution
def conv_kind(k, padding, fm=None, F=1):
    """special: 3x3, padding 1 on a dense square map that is replicated (or a
    single channel in and out); generic: any padding 0 <= P <= (k-1)/2 (the
    zero padding is realised by masking every tap whose neighbour falls
    outside the image, so the output fits the input's layout); padded: any
    larger padding, where the output is wider than the input, so the input
    is first re-laid out as the padded tensor X_p (pad_layout) and the
    generic schedule runs on it with P = 0."""
    if padding < 0:
        raise ValueError("negative padding")
    if k == 3 and padding == 1 and (fm is None or (
            fm.H == fm.W and fm.rs == fm.W and fm.cs == fm.W * fm.W and (fm.reps == 2 or (fm.C == 1 and F == 1)))):
        return "special"
    if padding <= (k - 1) // 2:
        return "generic"
    return "padded"


def padded_map(fm, P):
    """X_p's layout: (C, H + 2P, W + 2P) flattened densely, row stride
    W_p = W + 2P and channel block H_p W_p (section "Secure Advanced
    Convolution With Padding", equations for H_p and W_p)."""
    Hp, Wp = fm.H + 2 * P, fm.W + 2 * P
    return FMap(fm.C, Hp, Wp, Wp, Hp * Wp, 1)


def pad_plan(fm, P):
    """Steps that move X[c, y, x] from c cs + y rs + x to
    c cs' + (y + P) W_p + (x + P), zeros everywhere else in the blocks.

    The paper's reading: rows are spread apart with one rotation amount (the
    flattened rows are adjacent, so spreading them by 2P opens the left and
    right padding of neighbouring rows at once), channels are spread to their
    padded blocks, and one last rotation by W_p + P opens the top rows and
    the first row's left padding.  Here the row and channel spreads are
    masked chains (Horner with a single key each: rows key rs - W_p over
    the H rows, channels key cs - cs' over the C channels), one level each,
    so the layout needs three keys where the paper's per-channel rotations
    need C + 3.  Returns ([(step, count, key)], shift key, X_p's map): the
    channel step comes first when the blocks grow (rows then fit in them),
    the row step first otherwise; with neither needed one mask still clears
    whatever lies outside the image."""
    fp = padded_map(fm, P)
    rows = ("row", fm.H, fm.rs - fp.rs) if fm.rs != fp.rs else None
    chan = ("chan", fm.C, fm.cs - fp.cs) if fm.C > 1 and fm.cs != fp.cs else None
    if chan and rows:
        if (fm.H - 1) * fm.rs + fm.W <= fp.cs:
            steps = [chan, rows]
        elif (fm.H - 1) * fp.rs + fm.W <= fm.cs:
            steps = [rows, chan]
        else:
            raise NotImplementedError("the input layout leaves no room to re-lay out its rows")
    elif chan or rows:
        steps = [chan or rows]
    else:
        steps = [("clear", 1, 0)]
    return steps, -(P * fp.rs + P), fp


def pad_masks(fm, P, slots, bsgs=False):
    """Masks of pad_plan's steps, on the layout each step sees: channel t's
    image (t cs' or t cs + y rs + x), row t of every channel, or the whole
    image for the clearing step."""
    steps, _, fp = pad_plan(fm, P)
    if fm.C * fp.cs > slots:
        raise ValueError("the padded channels do not fit the slots")
    rs, cs = fm.rs, fm.cs
    out = []
    for step, n, key in steps:
        vecs = []
        for t in range(n):
            m = np.zeros(slots)
            for c in range(fm.C):
                for y in range(fm.H):
                    if (step == "chan" and c != t) or (step == "row" and y != t):
                        continue
                    base = c * cs + y * rs
                    m[base:base + fm.W] = 1.0
            vecs.append(m)
        out += chain_masks(vecs, key, bsgs) if n > 1 else vecs
        if step == "chan":
            cs = fp.cs
        elif step == "row":
            rs = fp.rs
    return out


def pad_keys(fm, P, bsgs=False):
    steps, shift, _ = pad_plan(fm, P)
    keys = {shift}
    for _, n, key in steps:
        keys |= masked_chain_keys(n, key, bsgs)
    return keys


def pad_layout(ev, x, fm, P, masks, bsgs=False):
    """X_p = Rot_{-(P W_p + P)}(chains of pad_plan applied to x); returns
    (X_p, its map).  Levels: one per step."""
    steps, shift, fp = pad_plan(fm, P)
    pos = 0
    for _, n, key in steps:
        x = masked_chain(ev, x, masks[pos:pos + n], n, key, bsgs)
        pos += n
    assert pos == len(masks)
    return ev.rot(x, shift), fp


def conv_taps(fm, k, padding):
    """Rotation of every tap (i, j), row-major: (i - P) rs + (j - P)."""
    return [(i - padding) * fm.rs + (j - padding) for i in range(k) for j in range(k)]


def conv_dims(fm, k, padding):
    """Stride-1 output size H + 2P - k + 1, W + 2P - k + 1."""
    return fm.H + 2 * padding - k + 1, fm.W + 2 * padding - k + 1


def conv_out_map(fm, F, k, stride, padding, slots):
    kind = conv_kind(k, padding, fm, F)
    if kind == "padded":
        return conv_out_map(padded_map(fm, padding), F, k, stride, 0, slots)
    if kind == "special":
        W = fm.W
        if stride == 1:
            reps = 2 if (fm.reps == 2 and 2 * F * W * W == slots) else 1
            return FMap(F, W, W, W, W * W, reps)
        Ho = (W + 2 - 3) // stride + 1
        return FMap(F, Ho, Ho, Ho, Ho * Ho, 1)
    H1, W1 = conv_dims(fm, k, padding)
    if stride == 1:
        return FMap(F, H1, W1, fm.rs, fm.cs, 1)
    Ho, Wo = (H1 - 1) // stride + 1, (W1 - 1) // stride + 1
    return FMap(F, Ho, Wo, Wo, Ho * Wo, 1)


def conv_plaintexts(fm, K, stride, padding, slots, bsgs=False, stride_log=False, stride_group=0):
    """Real vectors the convolution multiplies by, in the order the schedule
    (and the GPU library) consumes them: kernel vectors [f][tap], then masks."""
    F, C, k, _ = K.shape
    assert C == fm.C
    kind = conv_kind(k, padding, fm, F)
    if kind == "padded":
        kern, masks = conv_plaintexts(padded_map(fm, padding), K, stride, 0, slots, bsgs, stride_log, stride_group)
        return kern, pad_masks(fm, padding, slots, bsgs) + masks
    kern, masks = [], []
    if kind == "special":
        W = fm.W
        nm = special_masks(W, 1)
        for f in range(F):
            for tap in range(9):
                v = np.zeros(slots)
                dy, dx = tap // 3, tap % 3
                for b in range(fm.reps * C):
                    v[b * W * W:(b + 1) * W * W] = K[f, b % C, dy, dx] * nm[tap]
                kern.append(v)
        out1 = FMap(F, W, W, W, W * W, 2 if (fm.reps == 2 and 2 * F * W * W == slots) else 1)
        if F > 1 or C > 1:
            for f in range(F):
                m = np.zeros(slots)
                for r in range(out1.reps):
                    b = r * F + f
                    m[b * W * W:(b + 1) * W * W] = 1.0
                masks.append(m)
        if stride > 1:
            Ho = (W - 1) // stride + 1
            masks += strided_masks(FMap(F, W, W, W, W * W, 1), stride, Ho, Ho, 1.0, slots, bsgs, stride_log,
                                   stride_group)
    else:
        # tap (i, j) at output (y, x) reads input (y + i - P, x + j - P): the
        # kernel value where that neighbour is inside the image, 0 elsewhere
        H1, W1 = conv_dims(fm, k, padding)
        P = padding
        for f in range(F):
            for i in range(k):
                for j in range(k):
                    v = np.zeros(slots)
                    x0, x1 = max(0, P - j), min(W1, fm.W + P - j)
                    for c in range(C):
                        for y in range(H1):
                            if 0 <= y + i - P < fm.H and x0 < x1:
                                base = c * fm.cs + y * fm.rs
                                v[base + x0:base + x1] = K[f, c, i, j]
                    kern.append(v)
        if C > 1:
            m = np.zeros(slots)
            for y in range(H1):
                m[y * fm.rs:y * fm.rs + W1] = 1.0
            masks.append(m)
        if stride > 1:
            Ho, Wo = (H1 - 1) // stride + 1, (W1 - 1) // stride + 1
            masks += strided_masks(FMap(F, H1, W1, fm.rs, fm.cs, 1), stride, Ho, Wo, 1.0, slots, bsgs, stride_log,
                                   stride_group)
    return kern, masks


def logstep_ok(C):
    """The log-step channel sum applies to power-of-two channel counts."""
    return C > 1 and (C & (C - 1)) == 0


def channel_sum_keys(C, step, logstep):
    """Rotation keys of channel_sum."""
    if logstep and logstep_ok(C):
        return {step << t for t in range(C.bit_length() - 1)}
    return {step} if C > 1 else set()


def channel_sum(ev, A, C, step, logstep=False):
    """S = sum_{j < C} Rot_{j step}(A), the input-channel sum of a convolution.

    Chain (the paper's schedule, Algorithm 1's single key step): T <- Rot_step(T),
    S <- S + T, C - 1 key switches.  Log-step (C a power of two): S <- S +
    Rot_{2^t step}(S) for t < log2 C, log2 C key switches with keys 2^t step;
    Rot is linear and Rot_a Rot_b = Rot_{a+b}, so both give the same sum.
    """
    if logstep and logstep_ok(C):
        S, t = A, 1
        while t < C:
            S = ev.add(S, ev.rot(S, t * step))
            t *= 2
        return S
    S, T = A, A
    for _ in range(C - 1):
        T = ev.rot(T, step)
        S = ev.add(S, T)
    return S


def conv_rotations(fm, F, k, stride, padding, slots, logstep=False, bsgs=False, stride_log=False, stride_group=0):
    """Distinct rotation keys the schedule uses (the paper's per-layer index helper)."""
    kind = conv_kind(k, padding, fm, F)
    if kind == "padded":
        return sorted(pad_keys(fm, padding, bsgs) |
                      set(conv_rotations(padded_map(fm, padding), F, k, stride, 0, slots, logstep, bsgs, stride_log,
                                         stride_group)))
    keys = set()
    if kind == "special":
        W = fm.W
        keys |= {-W, W, -1, 1}
        keys |= channel_sum_keys(fm.C, W * W, logstep)
        if stride > 1:
            Ho = (W - 1) // stride + 1
            keys |= strided_keys(FMap(F, W, W, W, W * W, 1), stride, Ho, Ho, bsgs, stride_log, stride_group)
    else:
        keys |= {r for r in conv_taps(fm, k, padding) if r != 0}
        keys |= channel_sum_keys(fm.C, fm.cs, logstep)
        if F > 1:
            keys.add(-fm.cs)
        if stride > 1:
            H1, W1 = conv_dims(fm, k, padding)
            Ho, Wo = (H1 - 1) // stride + 1, (W1 - 1) // stride + 1
            keys |= strided_keys(FMap(F, H1, W1, fm.rs, fm.cs, 1), stride, Ho, Wo, bsgs, stride_log, stride_group)
    return sorted(keys)


def conv_bias_vector(fo, bias, slots):
    """The output channels' biases on the output layout fo: b_f at every
    position of channel f, in every replica (added after the convolution,
    the paper's "add the bias")."""
    v = np.zeros(slots)
    for r in range(fo.reps):
        for f in range(fo.C):
            for y in range(fo.H):
                base = (r * fo.C + f) * fo.cs + y * fo.rs
                v[base:base + fo.W] = bias[f]
    return v


def conv2d(ev, x, fm, F, k, stride, padding, kern, masks, slots, logstep=False, bsgs=False, bias=None,
           stride_log=False, stride_group=0):
    """The pinned convolution schedule (_conv2d_schedule), then the bias
    plaintext (conv_bias_vector, encoded at the output's scale and level)
    added when given."""
    y, fo = _conv2d_schedule(ev, x, fm, F, k, stride, padding, kern, masks, slots, logstep, bsgs, stride_log,
                             stride_group)
    if bias is not None:
        y = ev.add_plain(y, bias)
    return y, fo


def _conv2d_schedule(ev, x, fm, F, k, stride, padding, kern, masks, slots, logstep=False, bsgs=False,
                     stride_log=False, stride_group=0):
    """Pinned convolution schedule.

    special (k=3, P=1): r = Algorithm 1 rotations computed as three hoisted
      groups {-W, W, -1, 1} of x, {-1, 1} of r1, {-1, 1} of r7;
      A_f = RS(sum_tap r_tap (.) kv[f][tap]);
      C > 1 (replicated input): S_f = channel_sum(A_f, C, W^2), chained with
      the single key W^2 (C-1 key switches) or, with logstep and C a power of
      two, by doubling (log2 C key switches); Y = RS(sum_f S_f (.) blockmask_f);
      stride > 1: joint compaction of all channels (or, stride_group = g > 0,
      the paper's multi-channel pipeline: groups of g channels, merged).
    generic (0 <= P <= (k-1)/2): one hoisted group of the nonzero tap offsets
      (i - P) rs + (j - P); kernel vectors zero where a tap's neighbour lies
      in the padding; A_f = RS(sum r (.) kv); C > 1: channel_sum with step cs,
      then RS(. (.) block-0 mask); out-channels placed by a Horner chain with
      key -cs; stride > 1: joint compaction.
    padded (P > (k-1)/2): X_p = pad_layout(x) with the first pad masks, then
      the generic schedule with P = 0 on X_p's map and the remaining
      plaintexts.
    """
    kind = conv_kind(k, padding, fm, F)
    if kind == "padded":
        npad = len(pad_masks(fm, padding, slots, bsgs))
        xp, fp = pad_layout(ev, x, fm, padding, masks[:npad], bsgs)
        return _conv2d_schedule(ev, xp, fp, F, k, stride, 0, kern, masks[npad:], slots, logstep, bsgs, stride_log,
                                stride_group)
    C = fm.C
    if kind == "special":
        W = fm.W
        if fm.reps == 1 and (C > 1 or F > 1):
            raise NotImplementedError("special convolution with several channels needs a replicated input")
        if fm.reps == 2:
            assert 2 * C * W * W == slots
        g1 = ev.rot_hoisted(x, [-W, W, -1, 1])
        r1, r7, r3, r5 = g1
        r0, r2 = ev.rot_hoisted(r1, [-1, 1])
        r6, r8 = ev.rot_hoisted(r7, [-1, 1])
        taps = [r0, r1, r2, r3, x, r5, r6, r7, r8]
        sums = []
        for f in range(F):
            A = ev.rescale(mac(ev, taps, kern[9 * f:9 * f + 9]))
            sums.append(channel_sum(ev, A, C, W * W, logstep))
        mpos = 0
        if F > 1 or C > 1:
            y = ev.rescale(mac(ev, sums, masks[:F]))
            mpos = F
        else:
            y = sums[0]
        out1 = FMap(F, W, W, W, W * W, 2 if (fm.reps == 2 and 2 * F * W * W == slots) else 1)
        if stride == 1:
            return y, out1
        Ho = (W - 1) // stride + 1
        return strided(ev, y, FMap(F, W, W, W, W * W, 1), stride, Ho, Ho, masks[mpos:], bsgs, stride_log, stride_group)
    # generic
    offs = conv_taps(fm, k, padding)
    rot = iter(ev.rot_hoisted(x, [r for r in offs if r != 0]))
    taps = [x if r == 0 else next(rot) for r in offs]
    sums = []
    for f in range(F):
        A = ev.rescale(mac(ev, taps, kern[k * k * f:k * k * (f + 1)]))
        sums.append(channel_sum(ev, A, C, fm.cs, logstep))
    mpos = 0
    if C > 1:
        sums = [ev.mul_plain(s, masks[0]) for s in sums]
        mpos = 1
        y = horner(ev, lambda t: sums[t], F, -fm.cs)
    elif F > 1:
        acc = sums[F - 1]
        for t in range(F - 2, -1, -1):
            acc = ev.add(ev.rot(acc, -fm.cs), sums[t])
        y = acc
    else:
        y = sums[0]
    H1, W1 = conv_dims(fm, k, padding)
    if stride == 1:
        return y, FMap(F, H1, W1, fm.rs, fm.cs, 1)
    Ho, Wo = (H1 - 1) // stride + 1, (W1 - 1) // stride + 1
    return strided(ev, y, FMap(F, H1, W1, fm.rs, fm.cs, 1), stride, Ho, Wo, masks[mpos:], bsgs, stride_log,
                   stride_group)


# ===================================================================== pooling
def pool_whole_channel(fm, k):
    """The pooling special case: the window covers the whole (square, dense,
    power-of-two) channel, one output per channel, so the layer is the
    global schedule (channel sum, 1/k^2, each channel's first value
    gathered with one key)."""
    return (k > 0 and k == fm.H == fm.W and fm.rs == fm.W and fm.cs == fm.H * fm.W
            and fm.cs & (fm.cs - 1) == 0)


def avgpool_plaintexts(fm, k, stride, slots, bsgs=False, stride_log=False):
    if pool_whole_channel(fm, k):
        return gap_plaintexts(fm, slots, bsgs)
    H1, W1 = fm.H - k + 1, fm.W - k + 1
    Ho, Wo = (fm.H - k) // stride + 1, (fm.W - k) // stride + 1
    if stride == 1:
        m = np.zeros(slots)
        for c in range(fm.C):
            for y in range(H1):
                m[c * fm.cs + y * fm.rs:c * fm.cs + y * fm.rs + W1] = 1.0 / (k * k)
        return [m]
    return compaction_masks(FMap(fm.C, H1, W1, fm.rs, fm.cs, 1), stride, Ho, Wo, 1.0 / (k * k), slots, bsgs,
                            stride_log)


def avgpool_rotations(fm, k, stride, bsgs=False, stride_log=False):
    if pool_whole_channel(fm, k):
        return gap_rotations(fm, bsgs)
    keys = {i * fm.rs + j for i in range(k) for j in range(k) if (i, j) != (0, 0)}
    if stride > 1:
        H1, W1 = fm.H - k + 1, fm.W - k + 1
        Ho, Wo = (fm.H - k) // stride + 1, (fm.W - k) // stride + 1
        keys |= compaction_keys(FMap(fm.C, H1, W1, fm.rs, fm.cs, 1), stride, Ho, Wo, bsgs, stride_log)
    return sorted(keys)


def avgpool(ev, x, fm, k, stride, masks, bsgs=False, stride_log=False):
    """Window sum by one hoisted group of the k^2-1 offsets i rs + j, then the
    stride compaction with 1/k^2 folded into the column masks; a window over
    the whole channel is the global schedule (pool_whole_channel)."""
    if pool_whole_channel(fm, k):
        return gap(ev, x, fm, masks, bsgs)
    offs = [i * fm.rs + j for i in range(k) for j in range(k)]
    s = x
    for r in ev.rot_hoisted(x, offs[1:]):
        s = ev.add(s, r)
    H1, W1 = fm.H - k + 1, fm.W - k + 1
    if stride == 1:
        return ev.rescale(ev.mul_plain(s, masks[0])), FMap(fm.C, H1, W1, fm.rs, fm.cs, 1)
    Ho, Wo = (fm.H - k) // stride + 1, (fm.W - k) // stride + 1
    return compaction(ev, s, FMap(fm.C, H1, W1, fm.rs, fm.cs, 1), stride, Ho, Wo, masks, bsgs, stride_log)


def gap_plaintexts(fm, slots, bsgs=False):
    out = []
    for c in range(fm.C):
        m = np.zeros(slots)
        m[c * fm.cs] = 1.0 / (fm.H * fm.W)
        out.append(m)
    return chain_masks(out, fm.cs - 1, bsgs)


def gap_rotations(fm, bsgs=False):
    keys = {1 << t for t in range(int(math.log2(fm.cs)))}
    keys |= masked_chain_keys(fm.C, fm.cs - 1, bsgs)
    return sorted(keys)


def gap(ev, x, fm, masks, bsgs=False):
    """Global average pooling: S += Rot_{2^t}(S) for t < log2(cs) sums every
    channel block into its first slot; a Horner chain with key cs-1 and masks
    1/(H W) at c*cs gathers channel c into slot c."""
    assert fm.cs & (fm.cs - 1) == 0 and fm.rs == fm.W and fm.cs == fm.H * fm.W
    S = x
    for t in range(int(math.log2(fm.cs))):
        S = ev.add(S, ev.rot(S, 1 << t))
    y = masked_chain(ev, S, masks, fm.C, fm.cs - 1, bsgs)
    return y, FMap(fm.C, 1, 1, 1, 1, 1)


# ===================================================================== fully connected
def fc_plaintexts(Wm, slots):
    n_out, n_in = Wm.shape
    rows = []
    for k in range(n_out):
        v = np.zeros(slots)
        v[:n_in] = Wm[k]
        rows.append(v)
    e0 = np.zeros(slots)
    e0[0] = 1.0
    return rows, [e0]


def fc_rotations(n_in, n_out):
    return sorted({1 << t for t in range(int(math.log2(n_in)))} | ({-1} if n_out > 1 else set()))


def fc(ev, x, n_in, n_out, rows, masks):
    """Per output neuron: P_k = RS(x (.) W_k), log-step sum of n_in slots into
    slot 0; outputs consolidated by a Horner chain with key -1 over the
    e_0-masked sums (the paper's parameterised merging with one key)."""
    assert n_in & (n_in - 1) == 0
    sums = []
    for k in range(n_out):
        P = ev.rescale(ev.mul_plain(x, rows[k]))
        for t in range(int(math.log2(n_in))):
            P = ev.add(P, ev.rot(P, 1 << t))
        sums.append(P)
    return horner(ev, lambda k: ev.mul_plain(sums[k], masks[0]), n_out, -1)


def fc_diag_plaintexts(Wm, slots):
    """Diagonal form of the fully connected layer (n_out <= n_in, n_in a power
    of two): diagonal d holds W[j][(j + d) mod n_in] in slot j < n_out; with
    d = a B + b (bsgs_split) it is supplied rotated by -a B (np.roll by +a B)
    so that the inner sums of fc_diag need no further rotation."""
    n_out, n_in = Wm.shape
    assert n_in & (n_in - 1) == 0 and n_out <= n_in
    B, _ = bsgs_split(n_in)
    out = []
    for d in range(n_in):
        v = np.zeros(slots)
        for j in range(n_out):
            v[j] = Wm[j][(j + d) % n_in]
        out.append(np.roll(v, (d // B) * B))
    return out


def fc_diag_rotations(n_in):
    B, A = bsgs_split(n_in)
    return sorted({-n_in} | set(range(1, B)) | ({B} if A > 1 else set()))


def fc_diag(ev, x, n_in, n_out, diags):
    """y = W x with x in slots [0, n_in) (zeros in [n_in, 2 n_in) and in the
    top n_in slots): x~ = x + Rot_{-n_in}(x) makes slots [0, 2 n_in) periodic,
    so Rot_d(x~)[j] = x[(j + d) mod n_in] and y = sum_d diag_d . Rot_d(x~)
    (Halevi-Shoup).  Baby-step giant-step over d = a B + b: one hoisted group
    of Rot_b(x~), inner sums I_a = sum_b Rot_b(x~) . diag'_{aB+b} (diag'
    pre-rotated by -a B), acc = I_{A-1}; acc = Rot_B(acc) + I_a; one rescale.
    1 + (B - 1) + (A - 1) key switches, one level; y lands in slots
    [0, n_out), zeros elsewhere."""
    assert n_in & (n_in - 1) == 0 and n_out <= n_in
    B, A = bsgs_split(n_in)
    xt = ev.add(x, ev.rot(x, -n_in))
    baby = [xt] + (ev.rot_hoisted(xt, list(range(1, B))) if B > 1 else [])

    def inner(a):
        idx = range(a * B, min(n_in, a * B + B))
        return mac(ev, [baby[d - a * B] for d in idx], [diags[d] for d in idx])

    acc = inner(A - 1)
    for a in range(A - 2, -1, -1):
        acc = ev.add(ev.rot(acc, B), inner(a))
    return ev.rescale(acc)


# ===================================================================== polynomial activation
def relu_poly4(ev, x, delta):
    """p(x) = c0 + c1 x + c2 x^2 + c4 x^4 (RELU4) in three levels:
    x2 = RS(x*x); t = RS(x2 * c4) + c2; v = RS(x2 * t) (= c4 x^4 + c2 x^2);
    lin = RS(x * c1) with c1 encoded at sigma = s_v q / s_x so that it lands
    on v's level and scale (its tracked scale is set to s_v); p = v + lin + c0."""
    x2 = ev.rescale(ev.mul_relin(x, x))
    t = ev.add_const(ev.rescale(ev.mul_const(x2, RELU4[4], delta)), RELU4[2])
    v = ev.rescale(ev.mul_relin(ev.drop(x2, t.level), t))
    q = ev.modulus(v.level)  # the prime the next rescale divides by
    sigma = v.scale * q / x.scale
    lin = ev.rescale(ev.mul_const(ev.drop(x, v.level + 1), RELU4[1], sigma))
    lin = ev.with_scale(lin, v.scale)
    return ev.add_const(ev.add(v, lin), RELU4[0])


# ===================================================================== Chebyshev secure ReLU
def cheb_relu_coeffs(beta, degree=CHEB_DEGREE):
    """Chebyshev interpolant of f(z) = beta max(0, z) on [-1, 1] (the secure
    ReLU's function after the 1/beta input scaling): with the degree + 1
    nodes of the first kind z_k = cos(pi (k + 1/2) / (degree + 1)), the
    coefficients are c_j = 2 / (degree + 1) sum_k f(z_k) T_j(z_k) and
    f ~ c_0 / 2 + sum_{j >= 1} c_j T_j.  (The paper prints the node set
    garbled; these are the roots of T_{degree+1}, the standard choice.)
    f = beta z / 2 + beta |z| / 2: the odd part is interpolated exactly by
    T_1 and the even part only has even terms on the symmetric nodes, so
    c_1 = beta / 2 and every other odd coefficient is exactly zero."""
    n = degree + 1
    theta = np.pi * (np.arange(n) + 0.5) / n
    fz = beta * np.maximum(0.0, np.cos(theta))
    c = np.array([2.0 / n * float(np.sum(fz * np.cos(j * theta))) for j in range(n)])
    c[1::2] = 0.0
    if degree >= 1:
        c[1] = beta / 2.0
    return c


def cheb_relu_ref(x, beta, degree=CHEB_DEGREE):
    """FP64 value of the secure ReLU's polynomial at x: beta p(x / beta) with
    p the interpolant above divided by beta, i.e. chebval(x / beta) of the
    coefficients (c_0 halved)."""
    c = cheb_relu_coeffs(beta, degree).copy()
    c[0] /= 2.0
    return np.polynomial.chebyshev.chebval(np.asarray(x) / beta, c)


CHEB_BABY = 8  # baby-step bound of the evaluation: leaves have degree < 8


def cheb_series(coeffs):
    """Series coefficients a_j of f = sum a_j T_j (a_0 = c_0 / 2)."""
    a = np.array(coeffs, dtype=float)
    a[0] = a[0] / 2.0
    return a


def _trim(a):
    d = len(a) - 1
    while d > 0 and a[d] == 0.0:
        d -= 1
    return a[:d + 1]


def cheb_split(a, K):
    """Chebyshev division by T_K (K <= deg a < 2K): a = q T_K + r with
    T_{K+i} = 2 T_K T_i - T_{K-i}:  q_0 = a_K, q_i = 2 a_{K+i} (i >= 1);
    r_i = a_i - a_{2K-i} for 2K - deg <= i < K, r_i = a_i otherwise."""
    d = len(a) - 1
    q = np.zeros(d - K + 1)
    q[0] = a[K]
    for i in range(1, d - K + 1):
        q[i] = 2.0 * a[K + i]
    r = a[:K].copy()
    for i in range(2 * K - d, K):
        r[i] = a[i] - a[2 * K - i]
    return q, r


def cheb_tree(a):
    """The evaluation tree of a series: a leaf (degree < CHEB_BABY) or
    (K, quotient subtree, remainder subtree) with K = CHEB_BABY 2^m the
    largest such index not above the degree."""
    a = _trim(a)
    d = len(a) - 1
    if d < CHEB_BABY:
        return ("leaf", a)
    K = CHEB_BABY
    while 2 * K <= d:
        K *= 2
    q, r = cheb_split(a, K)
    return ("node", K, cheb_tree(q), cheb_tree(r))


def _tree_terms(t, acc):
    if t[0] == "leaf":
        acc |= {j for j in range(1, len(t[1])) if t[1][j] != 0.0}
        acc.add(1)
    else:
        acc.add(t[1])
        _tree_terms(t[2], acc)
        _tree_terms(t[3], acc)
    return acc


def _tree_nodes(t):
    return 0 if t[0] == "leaf" else 1 + _tree_nodes(t[2]) + _tree_nodes(t[3])


def cheb_terms(coeffs):
    """Chebyshev polynomials T_j (j >= 1) the evaluation computes, ascending:
    the leaves' terms with nonzero coefficients, T_1, the giant steps T_K and,
    recursively, the factors of the product rule (T_{2k} = 2 T_k^2 - 1,
    T_{2k+1} = 2 T_k T_{k+1} - T_1)."""
    need = set()
    stack = sorted(_tree_terms(cheb_tree(cheb_series(coeffs)), set()))
    while stack:
        j = stack.pop()
        if j in need:
            continue
        need.add(j)
        if j >= 2:
            stack.extend((j // 2,) if j % 2 == 0 else ((j - 1) // 2, (j + 1) // 2))
    return sorted(need)


def cheb_depth(j):
    """Multiplicative depth of T_j in the product rule (T_1: 0)."""
    return (j - 1).bit_length()


def _allowed(t, top):
    """Highest level a subtree can be evaluated onto when T_j sits at level top - depth(j)."""
    if t[0] == "leaf":
        js = [j for j in range(1, len(t[1])) if t[1][j] != 0.0] or [1]
        return min(top - cheb_depth(j) - 1 for j in js)
    K = t[1]
    return min(top - cheb_depth(K) - 1, _allowed(t[2], top) - 1, _allowed(t[3], top))


def cheb_plan(coeffs, masked):
    """(levels consumed, relinearizations) of cheb_eval."""
    tree = cheb_tree(cheb_series(coeffs))
    top = 0  # levels are relative to v = the (masked) input
    return int(masked) - _allowed(tree, top), len(cheb_terms(coeffs)) - 1 + _tree_nodes(tree)


def cheb_lift(ev, v, level, scale, c):
    """c v brought to `level` with tracked scale `scale`: drop v to level + 1,
    multiply by c encoded at sigma = scale q / s_v (q the prime the rescale
    divides by), rescale, and record `scale` (the product's, up to the
    rounding of sigma)."""
    q = ev.modulus(level)
    t = ev.rescale(ev.mul_const(ev.drop(v, level + 1), c, scale * q / v.scale))
    return ev.with_scale(t, scale)


def cheb_leaf(ev, a, T, level, scale):
    """A leaf sum_j a_j T_j + a_0 onto (level, scale) with one rescale: each
    T_j (j >= 1, a_j != 0, ascending; T_1 with 0 when there is none) dropped
    to level + 1 and multiplied by a_j encoded at sigma_j = scale q / s(T_j)
    (q the prime the rescale divides by), every product recorded at scale q
    (the same value up to the rounding of sigma_j), the products added,
    rescaled, recorded at `scale`, plus a_0."""
    q = ev.modulus(level)
    terms = [j for j in range(1, len(a)) if a[j] != 0.0] or [1]
    acc = None
    for j in terms:
        v = ev.drop(T[j], level + 1)
        p = ev.with_scale(ev.mul_const(v, a[j] if j < len(a) else 0.0, scale * q / v.scale), scale * q)
        acc = p if acc is None else ev.add(acc, p)
    return ev.add_const(ev.with_scale(ev.rescale(acc), scale), a[0])


def _cheb_node(ev, tree, T, level, scale):
    if tree[0] == "leaf":
        return cheb_leaf(ev, tree[1], T, level, scale)
    K, qt, rt = tree[1], tree[2], tree[3]
    sigma = scale * ev.modulus(level) / T[K].scale
    qc = _cheb_node(ev, qt, T, level + 1, sigma)
    p = ev.rescale(ev.mul_relin(qc, ev.drop(T[K], level + 1)))
    return ev.add(ev.with_scale(p, scale), _cheb_node(ev, rt, T, level, scale))


def cheb_eval(ev, x, coeffs, mask_pt, delta):
    """Secure ReLU (the paper's algorithm): v = RS(x * mask) when a 1/beta
    scale mask is given (beta > 1), else v = x; then f(v) = sum_j a_j T_j(v)
    (a_0 = c_0 / 2) by baby-step giant-step Chebyshev evaluation:
    * T_j for j in cheb_terms, ascending: factors aligned to the lower level,
      prod = RS(Relin(T_a T_b)), T_j = prod + prod - 1 (j even) or
      prod + prod + lift(v, -1) (j odd);
    * the series is split recursively by the giant steps T_K
      (a = q T_K + r, cheb_split) down to leaves of degree < CHEB_BABY;
    * every subtree is evaluated onto a given (level, scale): a leaf as
      RS(sum_j a_j T_j) plus a_0 (``cheb_leaf``: one rescale); a node as
      with_scale(RS(Relin(q' T_K)), scale) + r', with q' evaluated one level
      higher at scale * q_level / s(T_K) and r' at the node's own target;
    * the root target is the highest level every subtree allows."""
    v = ev.rescale(ev.mul_plain(x, mask_pt)) if mask_pt is not None else x
    T = {1: v}
    for j in cheb_terms(coeffs)[1:]:
        a, b = (j // 2, j // 2) if j % 2 == 0 else ((j - 1) // 2, (j + 1) // 2)
        lv = min(T[a].level, T[b].level)
        p = ev.rescale(ev.mul_relin(ev.drop(T[a], lv), ev.drop(T[b], lv)))
        p2 = ev.add(p, p)
        T[j] = ev.add_const(p2, -1.0) if j % 2 == 0 else ev.add(p2, cheb_lift(ev, v, p2.level, p2.scale, -1.0))
    tree = cheb_tree(cheb_series(coeffs))
    return _cheb_node(ev, tree, T, v.level + _allowed(tree, 0), delta)


def cheb_scale_mask(beta, n, slots):
    """GenerateScaleMask(beta, n): 1/beta on the first n slots, 0 elsewhere."""
    m = np.zeros(slots)
    m[:n] = 1.0 / beta
    return m
