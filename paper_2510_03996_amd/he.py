"""Python binding of the C ABI in ``include/he.h`` (argument marshalling only).

Every operation runs in the gfx950 HIP library ``libfheon_hip.so``; this
module only turns torch tensors (device memory) and the current HIP stream
into the raw pointers and sizes the C functions take.  There is no CPU
fallback: if the library cannot be loaded, every call raises.
"""
import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfheon_hip.so")

HE_OK = 0
ERRORS = {
    -1: "HE_EINVAL", -2: "HE_ENOKEY", -3: "HE_ELEVEL", -4: "HE_ESCALE",
    -5: "HE_ENOMEM", -6: "HE_EHIP", -7: "HE_EUNSUPPORTED",
}
KEY_RELIN = 0x7FFFFFFF
KEY_CONJ = 0x7FFFFFFE  # he_rotate with this id conjugates every slot
BOOT_MAX_ROTATIONS = 256
NTT_VARIANTS = 5
CHSUM_CHAIN, CHSUM_LOG = 0, 1  # he_ctx_conv_channel_sum modes
CHAIN_HORNER, CHAIN_BSGS = 0, 1  # he_ctx_mask_chains modes
STRIDE_EXTRACT, STRIDE_LOG = 0, 1  # he_ctx_striding modes
STRIDE_JOINT, STRIDE_GROUP_IN = 0, 1  # he_ctx_stride_groups modes
FC_ROWS, FC_DIAG = 0, 1  # he_ctx_fc_form modes
MAX_Q, MAX_P = 60, 16


class HEError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code
        self.name = ERRORS.get(code, "?")


class he_params(ctypes.Structure):
    _fields_ = [
        ("log_n", ctypes.c_int32), ("n_q", ctypes.c_int32), ("n_p", ctypes.c_int32), ("alpha", ctypes.c_int32),
        ("q_bits", ctypes.c_int32 * MAX_Q), ("p_bits", ctypes.c_int32 * MAX_P),
        ("q", ctypes.c_uint64 * MAX_Q), ("p", ctypes.c_uint64 * MAX_P),
    ]


class he_ct(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("level", ctypes.c_int32), ("cap", ctypes.c_int32),
                ("scale", ctypes.c_double)]


class he_pt(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("level", ctypes.c_int32), ("scale", ctypes.c_double)]


class he_fmap(ctypes.Structure):
    _fields_ = [("channels", ctypes.c_int32), ("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("row_stride", ctypes.c_int32), ("chan_stride", ctypes.c_int32), ("reps", ctypes.c_int32)]

    def key(self):
        return (self.channels, self.height, self.width, self.row_stride, self.chan_stride, self.reps)


def fmap(C, H, W, rs=None, cs=None, reps=1):
    rs = W if rs is None else rs
    cs = H * rs if cs is None else cs
    return he_fmap(C, H, W, rs, cs, reps)


class he_layer_plan(ctypes.Structure):
    _fields_ = [("n_kernel_pts", ctypes.c_int32), ("n_mask_pts", ctypes.c_int32), ("n_keys", ctypes.c_int32),
                ("rot_keys", ctypes.c_int32 * 64), ("levels", ctypes.c_int32), ("key_switches", ctypes.c_int32),
                ("out", he_fmap)]

    def keys(self):
        return [int(self.rot_keys[i]) for i in range(self.n_keys)]


class he_layer_desc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("log_n", ctypes.c_int32), ("mask_chains", ctypes.c_int32),
                ("fc_form", ctypes.c_int32), ("in_", he_fmap), ("out_ch", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("stride", ctypes.c_int32), ("padding", ctypes.c_int32), ("n_in", ctypes.c_int32),
                ("n_out", ctypes.c_int32), ("beta", ctypes.c_double), ("stride_mode", ctypes.c_int32),
                ("stride_groups", ctypes.c_int32), ("channel_sum", ctypes.c_int32)]


LAYER_CONV, LAYER_AVGPOOL, LAYER_FC, LAYER_CHEB_MASK = 0, 1, 2, 3


def _layer_desc(kind, log_n, fm=None, out_ch=0, kernel=0, stride=1, padding=0, n_in=0, n_out=0, beta=1.0,
                mask_chains=0, fc_form=0, stride_mode=0, stride_groups=0, channel_sum=0):
    return he_layer_desc(int(kind), int(log_n), int(mask_chains), int(fc_form), fm if fm is not None else he_fmap(),
                         int(out_ch), int(kernel), int(stride), int(padding), int(n_in), int(n_out), float(beta),
                         int(stride_mode), int(stride_groups), int(channel_sum))


def layer_rotations(kind, log_n, **options):
    """he_layer_rotations: a layer's plan (keys, plaintext counts, levels, key
    switches, output map) from its description, host only; options as for
    layer_plaintexts."""
    pl = he_layer_plan()
    _check(lib().he_layer_rotations(ctypes.byref(_layer_desc(kind, log_n, **options)), ctypes.byref(pl)))
    return pl


def layer_plaintexts(kind, log_n, weights=None, bias=None, fm=None, out_ch=0, kernel=0, stride=1, padding=0,
                     n_in=0, n_out=0, beta=1.0, mask_chains=0, fc_form=0, stride_mode=0, stride_groups=0,
                     channel_sum=0):
    """he_layer_plaintexts: the real slot vectors (float64 [count][N/2]) a
    layer consumes, in its plan's order (host only, no GPU needed)."""
    d = _layer_desc(kind, log_n, fm, out_ch, kernel, stride, padding, n_in, n_out, beta, mask_chains, fc_form,
                    stride_mode, stride_groups, channel_sum)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    b = None if bias is None else np.ascontiguousarray(bias, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    wp = w.ctypes.data_as(dp) if w is not None else None
    bp = b.ctypes.data_as(dp) if b is not None else None
    n = ctypes.c_int32()
    _check(lib().he_layer_plaintexts(ctypes.byref(d), wp, bp, None, 0, ctypes.byref(n)))
    out = np.zeros((n.value, (1 << int(log_n)) // 2))
    _check(lib().he_layer_plaintexts(ctypes.byref(d), wp, bp, out.ctypes.data_as(dp), n.value, ctypes.byref(n)))
    return out


class he_batch_desc(ctypes.Structure):
    _fields_ = [("n_items", ctypes.c_int32), ("level", ctypes.c_int32), ("in_scale", ctypes.c_double),
                ("pt_scale", ctypes.c_double), ("in_", ctypes.c_void_p), ("n_rot", ctypes.POINTER(ctypes.c_int32)),
                ("rots", ctypes.POINTER(ctypes.c_int32)), ("n_out", ctypes.POINTER(ctypes.c_int32)),
                ("pool", ctypes.c_void_p), ("n_pool", ctypes.c_int32), ("pool_level", ctypes.c_int32),
                ("pt_index", ctypes.POINTER(ctypes.c_int32)), ("out", ctypes.c_void_p)]


BATCH_GRAPH, BATCH_MAC4, BATCH_TUNE = 1, 2, 4
BATCH_MAC_VARIANTS = 5


class he_boot_desc(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("degree", ctypes.c_int32), ("level", ctypes.c_int32),
                ("double_angles", ctypes.c_int32), ("k_min", ctypes.c_double), ("delta", ctypes.c_double)]


def boot_desc(levels, degree, k_min, delta, level=0, double_angles=0):
    return he_boot_desc(int(levels), int(degree), int(level), int(double_angles), float(k_min), float(delta))


def boot_plan(log_n, levels, key_switches=False):
    """(rotation amounts, per-level plaintext counts: CoeffToSlot then
    SlotToCoeff[, key switches of both transforms]) of the bootstrapping
    transforms (host only)."""
    rots = (ctypes.c_int32 * BOOT_MAX_ROTATIONS)()
    nr, ks = ctypes.c_int32(), ctypes.c_int32()
    counts = (ctypes.c_int32 * max(1, 2 * levels))()
    _check(lib().he_boot_plan(int(log_n), int(levels), rots, ctypes.byref(nr), counts, ctypes.byref(ks)))
    out = (list(rots[: nr.value]), list(counts))
    return out + (ks.value,) if key_switches else out


def boot_diagonals(log_n, levels, inverse):
    """Complex slot vectors of every plaintext of one transform, in
    consumption order (host only): a list of numpy complex arrays."""
    import numpy as np

    _, counts = boot_plan(log_n, levels)
    k = sum(counts[:levels]) if inverse else sum(counts[levels:])
    n = 1 << (log_n - 1)
    re = np.zeros(k * n)
    im = np.zeros(k * n)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib().he_boot_diagonals(int(log_n), int(levels), 1 if inverse else 0, re.ctypes.data_as(dp),
                                   im.ctypes.data_as(dp), re.size))
    return [(re[i * n:(i + 1) * n] + 1j * im[i * n:(i + 1) * n]) for i in range(k)]


def boot_mod_coeffs(K, degree, double_angles=0):
    cf = (ctypes.c_double * (degree + 1))()
    _check(lib().he_boot_mod_coeffs(float(K), int(degree), int(double_angles), cf))
    return list(cf)


def batch_mac_select(v):
    """HE_BATCH_MAC_SELECT(v): run the batched MAC as variant v (0..4)."""
    return (int(v) + 1) << 8

_lib = None


def lib():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libfheon_hip.so is not built; run python -m paper_2510_03996_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, c_int, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int, ctypes.c_size_t
        P = ctypes.POINTER
        sig = {
            "he_ctx_create": [P(he_params), c_int, P(vp)],
            "he_ctx_destroy": [vp],
            "he_ctx_moduli": [vp, P(ctypes.c_uint64), c_int],
            "he_ctx_info": [vp, P(i32), P(i32), P(i32), P(i32)],
            "he_key_upload": [vp, i32, vp, sz, c_int, vp],
            "he_key_evict": [vp, i32],
            "he_key_count": [vp],
            "he_ntt": [vp, vp, c_int, c_int, c_int, vp],
            "he_rotate": [vp, P(he_ct), i32, P(he_ct), vp],
            "he_rotate_noalloc": [vp, P(he_ct), i32, P(he_ct), vp],
            "he_rotate_hoisted": [vp, P(he_ct), P(i32), c_int, P(he_ct), vp],
            "he_mul_plain": [vp, P(he_ct), P(he_pt), P(he_ct), c_int, vp],
            "he_add": [vp, P(he_ct), P(he_ct), P(he_ct), vp],
            "he_sub": [vp, P(he_ct), P(he_ct), P(he_ct), vp],
            "he_add_plain": [vp, P(he_ct), P(he_pt), P(he_ct), vp],
            "he_rescale": [vp, P(he_ct), P(he_ct), vp],
            "he_drop_level": [vp, P(he_ct), c_int, P(he_ct), vp],
            "he_mul_relin": [vp, P(he_ct), P(he_ct), P(he_ct), vp],
            "he_relin": [vp, vp, c_int, ctypes.c_double, P(he_ct), vp],
            "he_mul_const": [vp, P(he_ct), ctypes.c_double, ctypes.c_double, P(he_ct), vp],
            "he_add_const": [vp, P(he_ct), ctypes.c_double, P(he_ct), vp],
            "he_conv2d_plan": [vp, P(he_fmap), c_int, c_int, c_int, c_int, P(he_layer_plan)],
            "he_conv2d": [vp, P(he_ct), P(he_fmap), c_int, c_int, c_int, c_int, P(he_pt), c_int, P(he_pt), c_int,
                          P(he_pt), P(he_ct), P(he_fmap), vp],
            "he_layer_plaintexts": [P(he_layer_desc), P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_double),
                                    ctypes.c_size_t, P(i32)],
            "he_layer_rotations": [P(he_layer_desc), P(he_layer_plan)],
            "he_avgpool_plan": [vp, P(he_fmap), c_int, c_int, P(he_layer_plan)],
            "he_avgpool": [vp, P(he_ct), P(he_fmap), c_int, c_int, P(he_pt), c_int, P(he_ct), P(he_fmap), vp],
            "he_fc_plan": [vp, c_int, c_int, P(he_layer_plan)],
            "he_fc": [vp, P(he_ct), c_int, c_int, P(he_pt), P(he_pt), P(he_pt), P(he_ct), vp],
            "he_poly4": [vp, P(he_ct), P(ctypes.c_double), ctypes.c_double, P(he_ct), vp],
            "he_cheb": [vp, P(he_ct), P(he_pt), P(ctypes.c_double), c_int, ctypes.c_double, P(he_ct), vp],
            "he_cheb_plan": [P(ctypes.c_double), c_int, c_int, P(i32), P(i32)],
            "he_cheb_relu_coeffs": [ctypes.c_double, c_int, P(ctypes.c_double)],
            "he_batch_create": [vp, P(he_batch_desc), c_int, P(vp)],
            "he_batch_run": [vp, vp],
            "he_batch_run_plain": [vp, vp],
            "he_batch_info": [vp, P(i32), P(i32), P(i32), P(ctypes.c_double)],
            "he_batch_destroy": [vp],
            "he_batch_tuning": [vp, P(i32), P(i32), P(ctypes.c_float), i32],
            "he_lane_reserve": [vp, vp, c_int],
            "he_lane_release": [vp, vp],
            "he_ctx_ntt_tuning": [vp, P(i32), P(ctypes.c_float)],
            "he_ctx_conv_tuning": [vp, P(i32), P(ctypes.c_float)],
            "he_ntt_variant": [c_int, P(i32), P(i32)],
            "he_ctx_ntt_select": [vp, P(i32)],
            "he_ctx_conv_channel_sum": [vp, i32],
            "he_ctx_mask_chains": [vp, i32],
            "he_ctx_striding": [vp, i32],
            "he_ctx_stride_groups": [vp, i32],
            "he_ctx_fc_form": [vp, i32],
            "he_ctx_layer_streams": [vp, i32],
            "he_key_host_register": [vp, i32, P(ctypes.c_uint64), sz],
            "he_key_cache_limit": [vp, sz],
            "he_key_prefetch": [vp, P(i32), c_int, vp],
            "he_key_cache_stats": [vp, P(sz), P(ctypes.c_int64), P(ctypes.c_int64)],
            "he_mul_i": [vp, P(he_ct), c_int, P(he_ct), vp],
            "he_mac_plain": [vp, P(he_ct), P(he_pt), c_int, P(he_ct), c_int, vp],
            "he_mod_raise": [vp, P(he_ct), c_int, P(he_ct), vp],
            "he_boot_plan": [i32, i32, P(i32), P(i32), P(i32), P(i32)],
            "he_boot_diagonals": [i32, i32, i32, P(ctypes.c_double), P(ctypes.c_double), sz],
            "he_boot_mod_coeffs": [ctypes.c_double, i32, i32, P(ctypes.c_double)],
            "he_boot_scales": [vp, P(he_boot_desc), P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_double),
                               P(ctypes.c_double)],
            "he_bootstrap": [vp, P(he_ct), P(he_boot_desc), P(he_pt), P(he_pt), P(ctypes.c_double), P(he_ct), vp],
            "he_capture_begin": [vp, vp],
            "he_capture_end": [vp, vp, P(vp)],
            "he_graph_launch": [vp, vp],
            "he_graph_destroy": [vp],
            "he_profile_begin": [vp],
            "he_profile_end": [vp, ctypes.c_char_p, sz],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = c_int
        L.he_last_error.restype = ctypes.c_char_p
        L.he_last_error.argtypes = []
        L.he_key_bytes.restype = ctypes.c_size_t
        L.he_key_bytes.argtypes = [vp]
        L.he_lane_bytes.restype = ctypes.c_size_t
        L.he_lane_bytes.argtypes = [vp, c_int]
        _lib = L
    return _lib


def _check(rc):
    if rc < 0:
        raise HEError(rc, lib().he_last_error().decode())
    return rc


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    assert t.is_cuda and t.is_contiguous() and t.dtype == torch.int64
    return ctypes.c_void_p(t.data_ptr())


class Ciphertext:
    """A device ciphertext: int64 tensor [2][cap][N] holding uint64 residues."""

    def __init__(self, data, level, scale):
        self.data = data
        self.level = int(level)
        self.scale = float(scale)

    @property
    def cap(self):
        return self.data.shape[1]

    def c(self):
        return he_ct(ctypes.c_void_p(self.data.data_ptr()), self.level, self.cap, self.scale)

    def update(self, s):
        self.level, self.scale = s.level, s.scale

    def numpy(self):
        """uint64 [2][level][N] copy on the host."""
        return self.data[:, : self.level].cpu().numpy().view(np.uint64)


class Plaintext:
    def __init__(self, data, scale):
        self.data = data  # int64 [level][N]
        self.scale = float(scale)

    @property
    def level(self):
        return self.data.shape[0]

    def c(self):
        return he_pt(ctypes.c_void_p(self.data.data_ptr()), self.level, self.scale)


def _pts(pts):
    arr = (he_pt * max(1, len(pts)))(*[p.c() for p in pts])
    return arr


def to_device(arr_u64, device="cuda"):
    """uint64 numpy array -> int64 device tensor with the same bits."""
    a = np.ascontiguousarray(arr_u64, dtype=np.uint64)
    return torch.from_numpy(a.view(np.int64)).to(device)


class Context:
    """A library context (moduli, tables, resident keys, workspace)."""

    def __init__(self, log_n, q_bits, p_bits, alpha, device=0, primes=None):
        p = he_params()
        p.log_n, p.n_q, p.n_p, p.alpha = log_n, len(q_bits), len(p_bits), alpha
        for i, b in enumerate(q_bits):
            p.q_bits[i] = b
        for i, b in enumerate(p_bits):
            p.p_bits[i] = b
        if primes is not None:
            for i, v in enumerate(primes[0]):
                p.q[i] = v
            for i, v in enumerate(primes[1]):
                p.p[i] = v
        h = ctypes.c_void_p()
        _check(lib().he_ctx_create(ctypes.byref(p), device, ctypes.byref(h)))
        self.h = h
        self.log_n, self.n = log_n, 1 << log_n
        self.L, self.K, self.alpha = len(q_bits), len(p_bits), alpha
        self.device = torch.device("cuda", device)
        buf = (ctypes.c_uint64 * (self.L + self.K))()
        _check(lib().he_ctx_moduli(h, buf, self.L + self.K))
        self.moduli = [int(x) for x in buf]

    def close(self):
        if self.h:
            torch.cuda.synchronize()
            lib().he_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def dnum(self):
        return -(-self.L // self.alpha)

    def key_bytes(self):
        return lib().he_key_bytes(self.h)

    # ---- buffers
    def new_ct(self, cap=None):
        cap = cap or self.L
        return Ciphertext(torch.empty((2, cap, self.n), dtype=torch.int64, device=self.device), 0, 0.0)

    def ct_from_numpy(self, data_u64, scale, cap=None):
        d = np.asarray(data_u64, dtype=np.uint64)
        level = d.shape[1]
        cap = cap or level
        t = torch.zeros((2, cap, self.n), dtype=torch.int64, device=self.device)
        t[:, :level] = to_device(d, self.device)
        return Ciphertext(t, level, scale)

    def pt_from_numpy(self, data_u64, scale):
        return Plaintext(to_device(data_u64, self.device), scale)

    # ---- keys
    def key_upload(self, key_id, key, stream=None):
        if isinstance(key, np.ndarray):
            k = np.ascontiguousarray(key, dtype=np.uint64)
            _check(lib().he_key_upload(self.h, key_id, ctypes.c_void_p(k.ctypes.data), k.nbytes, 0, _stream(stream)))
        else:
            _check(lib().he_key_upload(self.h, key_id, _ptr(key), key.numel() * 8, 1, _stream(stream)))

    def key_evict(self, key_id):
        _check(lib().he_key_evict(self.h, key_id))

    def key_host_register(self, key_id, key):
        """Register a key by a host copy (loaded into device memory on demand)."""
        k = np.ascontiguousarray(np.asarray(key), dtype=np.uint64)
        _check(lib().he_key_host_register(self.h, int(key_id), k.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                          k.nbytes))

    def key_cache_limit(self, device_bytes):
        _check(lib().he_key_cache_limit(self.h, int(device_bytes)))

    def key_prefetch(self, key_ids, stream=None):
        ids = (ctypes.c_int32 * len(key_ids))(*[int(x) for x in key_ids])
        _check(lib().he_key_prefetch(self.h, ids, len(key_ids), _stream(stream)))

    def key_cache_stats(self):
        r, lo, ev = ctypes.c_size_t(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().he_key_cache_stats(self.h, ctypes.byref(r), ctypes.byref(lo), ctypes.byref(ev)))
        return {"resident_bytes": r.value, "loads": lo.value, "evictions": ev.value}

    def key_count(self):
        return lib().he_key_count(self.h)

    # ---- ops
    def ntt(self, poly, first_limb=0, inverse=False, stream=None):
        _check(lib().he_ntt(self.h, _ptr(poly), poly.shape[0], first_limb, 1 if inverse else 0, _stream(stream)))

    def rotate(self, ct, r, out=None, stream=None):
        out = out or self.new_ct(ct.level)
        a, o = ct.c(), out.c()
        _check(lib().he_rotate(self.h, ctypes.byref(a), int(r), ctypes.byref(o), _stream(stream)))
        out.update(o)
        return out

    def rotate_noalloc(self, ct, r, out, stream=None):
        """he_rotate with the key-switch workspace in the library's static
        device array (allocates nothing; out must be preallocated)."""
        a, o = ct.c(), out.c()
        _check(lib().he_rotate_noalloc(self.h, ctypes.byref(a), int(r), ctypes.byref(o), _stream(stream)))
        out.update(o)
        return out

    def rotate_hoisted(self, ct, rs, outs=None, stream=None):
        outs = outs or [self.new_ct(ct.level) for _ in rs]
        a = ct.c()
        arr = (he_ct * len(rs))(*[o.c() for o in outs])
        rr = (ctypes.c_int32 * len(rs))(*[int(r) for r in rs])
        _check(lib().he_rotate_hoisted(self.h, ctypes.byref(a), rr, len(rs), arr, _stream(stream)))
        for o, s in zip(outs, arr):
            o.update(s)
        return outs

    def mul_plain(self, ct, pt, out=None, accumulate=False, stream=None):
        out = out or self.new_ct(ct.level)
        a, p, o = ct.c(), pt.c(), out.c()
        _check(lib().he_mul_plain(self.h, ctypes.byref(a), ctypes.byref(p), ctypes.byref(o), int(accumulate),
                                  _stream(stream)))
        out.update(o)
        return out

    def _binary(self, fn, a, b, out, stream):
        out = out or self.new_ct(a.level)
        x, y, o = a.c(), b.c(), out.c()
        _check(fn(self.h, ctypes.byref(x), ctypes.byref(y), ctypes.byref(o), _stream(stream)))
        out.update(o)
        return out

    def add(self, a, b, out=None, stream=None):
        return self._binary(lib().he_add, a, b, out, stream)

    def sub(self, a, b, out=None, stream=None):
        return self._binary(lib().he_sub, a, b, out, stream)

    def mul_relin(self, a, b, out=None, stream=None):
        return self._binary(lib().he_mul_relin, a, b, out, stream)

    def add_plain(self, a, pt, out=None, stream=None):
        out = out or self.new_ct(a.level)
        x, p, o = a.c(), pt.c(), out.c()
        _check(lib().he_add_plain(self.h, ctypes.byref(x), ctypes.byref(p), ctypes.byref(o), _stream(stream)))
        out.update(o)
        return out

    def rescale(self, ct, out=None, stream=None):
        out = out or self.new_ct(ct.cap)
        a, o = ct.c(), out.c()
        _check(lib().he_rescale(self.h, ctypes.byref(a), ctypes.byref(o), _stream(stream)))
        out.update(o)
        return out

    def drop_level(self, ct, level, out=None, stream=None):
        out = out or self.new_ct(ct.cap)
        a, o = ct.c(), out.c()
        _check(lib().he_drop_level(self.h, ctypes.byref(a), level, ctypes.byref(o), _stream(stream)))
        out.update(o)
        return out

    def relin(self, d, level, scale, out=None, stream=None):
        out = out or self.new_ct(level)
        o = out.c()
        _check(lib().he_relin(self.h, _ptr(d), level, scale, ctypes.byref(o), _stream(stream)))
        out.update(o)
        return out

    # ---- constants
    def mul_const(self, ct, c, scale, out=None, stream=None):
        out = out or self.new_ct(ct.cap)
        a, o = ct.c(), out.c()
        _check(lib().he_mul_const(self.h, ctypes.byref(a), float(c), float(scale), ctypes.byref(o), _stream(stream)))
        out.update(o)
        return out

    def add_const(self, ct, c, out=None, stream=None):
        out = out or self.new_ct(ct.cap)
        a, o = ct.c(), out.c()
        _check(lib().he_add_const(self.h, ctypes.byref(a), float(c), ctypes.byref(o), _stream(stream)))
        out.update(o)
        return out

    # ---- layers
    def conv2d_plan(self, fm, out_ch, kernel, stride, padding):
        pl = he_layer_plan()
        _check(lib().he_conv2d_plan(self.h, ctypes.byref(fm), out_ch, kernel, stride, padding, ctypes.byref(pl)))
        return pl

    def conv2d(self, ct, fm, out_ch, kernel, stride, padding, kernel_pts, mask_pts, out=None, stream=None,
               bias_pt=None):
        out = out or self.new_ct(ct.cap)
        a, o, om = ct.c(), out.c(), he_fmap()
        b = ctypes.byref(bias_pt.c()) if bias_pt is not None else None
        _check(lib().he_conv2d(self.h, ctypes.byref(a), ctypes.byref(fm), out_ch, kernel, stride, padding,
                               _pts(kernel_pts), len(kernel_pts), _pts(mask_pts), len(mask_pts), b, ctypes.byref(o),
                               ctypes.byref(om), _stream(stream)))
        out.update(o)
        return out, om

    def avgpool_plan(self, fm, kernel, stride):
        pl = he_layer_plan()
        _check(lib().he_avgpool_plan(self.h, ctypes.byref(fm), kernel, stride, ctypes.byref(pl)))
        return pl

    def avgpool(self, ct, fm, kernel, stride, mask_pts, out=None, stream=None):
        out = out or self.new_ct(ct.cap)
        a, o, om = ct.c(), out.c(), he_fmap()
        _check(lib().he_avgpool(self.h, ctypes.byref(a), ctypes.byref(fm), kernel, stride, _pts(mask_pts),
                                len(mask_pts), ctypes.byref(o), ctypes.byref(om), _stream(stream)))
        out.update(o)
        return out, om

    def fc_plan(self, n_in, n_out):
        pl = he_layer_plan()
        _check(lib().he_fc_plan(self.h, n_in, n_out, ctypes.byref(pl)))
        return pl

    def fc(self, ct, n_in, n_out, weight_pts, mask_pts, bias_pt=None, out=None, stream=None):
        out = out or self.new_ct(ct.cap)
        a, o = ct.c(), out.c()
        b = ctypes.byref(bias_pt.c()) if bias_pt is not None else None
        _check(lib().he_fc(self.h, ctypes.byref(a), n_in, n_out, _pts(weight_pts), _pts(mask_pts), b,
                           ctypes.byref(o), _stream(stream)))
        out.update(o)
        return out

    def poly4(self, ct, coeffs, delta, out=None, stream=None):
        out = out or self.new_ct(ct.cap)
        a, o = ct.c(), out.c()
        cf = (ctypes.c_double * 5)(*[float(x) for x in coeffs])
        _check(lib().he_poly4(self.h, ctypes.byref(a), cf, float(delta), ctypes.byref(o), _stream(stream)))
        out.update(o)
        return out

    def cheb(self, ct, coeffs, delta, scale_mask=None, out=None, stream=None):
        """Secure ReLU / Chebyshev series (he_cheb); coeffs = c_0..c_D."""
        levels, _ = cheb_plan(coeffs, scale_mask is not None)
        out = out or self.new_ct(max(ct.level - levels, 1))
        a, o = ct.c(), out.c()
        cf = (ctypes.c_double * len(coeffs))(*[float(x) for x in coeffs])
        m = ctypes.byref(scale_mask.c()) if scale_mask is not None else None
        _check(lib().he_cheb(self.h, ctypes.byref(a), m, cf, len(coeffs) - 1, float(delta), ctypes.byref(o),
                             _stream(stream)))
        out.update(o)
        return out

    def mac_plain(self, cts, pts, out=None, accumulate=False, stream=None):
        """out (+)= sum_t cts[t] (.) pts[t] in one pass."""
        out = out or self.new_ct(cts[0].cap)
        arr = (he_ct * len(cts))(*[c.c() for c in cts])
        o = out.c()
        _check(lib().he_mac_plain(self.h, arr, _pts(pts), len(cts), ctypes.byref(o), 1 if accumulate else 0,
                                  _stream(stream)))
        out.update(o)
        return out

    def capture_begin(self, stream):
        """Start recording the library calls issued on `stream` (not the
        default stream) into a graph (he_capture_begin's rules apply)."""
        _check(lib().he_capture_begin(self.h, _stream(stream)))

    def capture_end(self, stream):
        g = ctypes.c_void_p()
        _check(lib().he_capture_end(self.h, _stream(stream), ctypes.byref(g)))
        return Graph(g)

    def mul_i(self, ct, sign, out=None, stream=None):
        out = out or self.new_ct(ct.cap)
        a, o = ct.c(), out.c()
        _check(lib().he_mul_i(self.h, ctypes.byref(a), int(sign), ctypes.byref(o), _stream(stream)))
        out.update(o)
        return out

    def mod_raise(self, ct, level, out=None, stream=None):
        out = out or self.new_ct(level)
        a, o = ct.c(), out.c()
        _check(lib().he_mod_raise(self.h, ctypes.byref(a), int(level), ctypes.byref(o), _stream(stream)))
        out.update(o)
        return out

    def boot_scales(self, desc):
        """(K, raise scale, CoeffToSlot scales, SlotToCoeff scales)."""
        K, rs = ctypes.c_double(), ctypes.c_double()
        cs = (ctypes.c_double * desc.levels)()
        ss = (ctypes.c_double * desc.levels)()
        _check(lib().he_boot_scales(self.h, ctypes.byref(desc), ctypes.byref(K), ctypes.byref(rs), cs, ss))
        return K.value, rs.value, list(cs), list(ss)

    def bootstrap(self, ct, desc, cts_pts, stc_pts, coeffs, out=None, stream=None):
        out = out or self.new_ct()
        a, o = ct.c(), out.c()
        cf = (ctypes.c_double * len(coeffs))(*[float(x) for x in coeffs])
        _check(lib().he_bootstrap(self.h, ctypes.byref(a), ctypes.byref(desc), _pts(cts_pts), _pts(stc_pts), cf,
                                  ctypes.byref(o), _stream(stream)))
        out.update(o)
        return out

    def ntt_tuning(self):
        nv = NTT_VARIANTS
        var = (ctypes.c_int32 * 4)()
        us = (ctypes.c_float * (nv * 4))()
        _check(lib().he_ctx_ntt_tuning(self.h, var, us))
        shapes = []
        for v in range(nv):
            t, e = ctypes.c_int32(), ctypes.c_int32()
            _check(lib().he_ntt_variant(v, ctypes.byref(t), ctypes.byref(e)))
            shapes.append("%dx%d" % (t.value, e.value))
        return {"bucket_max_limbs": [8, 16, 32, "more"], "variant_tile_x_per_thread": [shapes[v] for v in var],
                "us_fwd_inv": {shapes[v]: [round(us[v * 4 + i], 2) for i in range(4)] for v in range(nv)}}

    def conv_tuning(self):
        """Basis-conversion workgroup targets chosen at creation (ModUp, ModDown)
        and the timings of the candidates."""
        tg = (ctypes.c_int32 * 2)()
        us = (ctypes.c_float * 8)()
        _check(lib().he_ctx_conv_tuning(self.h, tg, us))
        cand = [512, 768, 1024, 1536]
        return {"modup_target": tg[0], "moddown_target": tg[1],
                "us": {"modup": dict(zip(cand, [round(us[i], 2) for i in range(4)])),
                       "moddown": dict(zip(cand, [round(us[4 + i], 2) for i in range(4)]))}}

    def ntt_select(self, variants):
        """Pin the NTT variant of each batch-size bucket (4 entries)."""
        _check(lib().he_ctx_ntt_select(self.h, (ctypes.c_int32 * 4)(*[int(v) for v in variants])))

    def conv_channel_sum(self, mode):
        """Input-channel sum of later conv2d plans and calls: CHSUM_CHAIN (the
        paper's single-key chain) or CHSUM_LOG (doubling, log2 C keys)."""
        _check(lib().he_ctx_conv_channel_sum(self.h, int(mode)))

    def mask_chains(self, mode):
        """Masked rotation chains of later layer plans and calls: CHAIN_HORNER
        or CHAIN_BSGS (baby-step giant-step; masks pre-rotated by the caller)."""
        _check(lib().he_ctx_mask_chains(self.h, int(mode)))

    def striding(self, mode):
        """Column step of the stride compaction of later conv2d / avgpool plans
        and calls: STRIDE_EXTRACT (one chain over the columns) or STRIDE_LOG
        (ceil(log2 Wo) two-term steps, the paper's second approach)."""
        _check(lib().he_ctx_striding(self.h, int(mode)))

    def stride_groups(self, mode):
        """Output-channel grouping of later strided conv2d plans and calls:
        STRIDE_JOINT (all channels at once) or STRIDE_GROUP_IN (the paper's
        groups of the layer's input channels, merged with one more key)."""
        _check(lib().he_ctx_stride_groups(self.h, int(mode)))

    def fc_form(self, mode):
        """Form of later fc plans and calls: FC_ROWS (per neuron) or FC_DIAG
        (diagonal, baby-step giant-step; weight_pts are the rotated diagonals)."""
        _check(lib().he_ctx_fc_form(self.h, int(mode)))

    def layer_streams(self, n):
        """Streams (1..8, default 2) a convolution's output channels and a
        hoisted set's key switches are spread over: the caller's stream plus
        n - 1 helper streams of it; results do not depend on n."""
        _check(lib().he_ctx_layer_streams(self.h, int(n)))

    def ntt_variants(self):
        var = (ctypes.c_int32 * 4)()
        _check(lib().he_ctx_ntt_tuning(self.h, var, None))
        return list(var)

    # ---- lanes
    def lane_reserve(self, stream, n_ct_buffers):
        _check(lib().he_lane_reserve(self.h, _stream(stream), n_ct_buffers))

    def lane_release(self, stream):
        _check(lib().he_lane_release(self.h, _stream(stream)))

    def lane_bytes(self, n_ct_buffers):
        return lib().he_lane_bytes(self.h, n_ct_buffers)

    # ---- measurement
    def profile_begin(self):
        _check(lib().he_profile_begin(self.h))

    def profile_end(self):
        import json

        buf = ctypes.create_string_buffer(1 << 16)
        n = _check(lib().he_profile_end(self.h, buf, len(buf)))
        return json.loads(buf.value[:n].decode())


def cheb_plan(coeffs, masked):
    """(levels consumed, relinearizations) of Context.cheb (host only)."""
    cf = (ctypes.c_double * len(coeffs))(*[float(x) for x in coeffs])
    lv, rl = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().he_cheb_plan(cf, len(coeffs) - 1, 1 if masked else 0, ctypes.byref(lv), ctypes.byref(rl)))
    return lv.value, rl.value


def cheb_relu_coeffs(beta, degree=59):
    """Chebyshev interpolation coefficients of beta max(0, z) on [-1, 1] (host only)."""
    cf = (ctypes.c_double * (degree + 1))()
    _check(lib().he_cheb_relu_coeffs(float(beta), int(degree), cf))
    return list(cf)


class Graph:
    """A captured sequence of library calls (he_graph)."""

    def __init__(self, handle):
        self.h = handle

    def launch(self, stream=None):
        _check(lib().he_graph_launch(self.h, _stream(stream)))

    def close(self):
        if self.h:
            lib().he_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Batched hoisted-rotation multiply-accumulate (see he_batch_create).

    inp: int64 device tensor [B][2][l][N]; rot_sets: list of B lists of
    rotation amounts; n_outs: list of B output counts; pool: int64 device
    tensor [P][pool_level][N]; pt_index: list of B lists (n_out x n_rot,
    o-major) of pool indices; out: int64 device tensor [sum n_outs][2][l-1][N].
    """

    def __init__(self, ctx, inp, level, in_scale, rot_sets, n_outs, pool, pt_scale, pt_index, out, flags=0):
        self.ctx = ctx
        self.keep = (inp, pool, out)
        B = len(rot_sets)
        self._n_rot = (ctypes.c_int32 * B)(*[len(r) for r in rot_sets])
        flat = [int(x) for r in rot_sets for x in r]
        self._rots = (ctypes.c_int32 * len(flat))(*flat)
        self._n_out = (ctypes.c_int32 * B)(*[int(m) for m in n_outs])
        fi = [int(x) for lst in pt_index for x in lst]
        self._pti = (ctypes.c_int32 * len(fi))(*fi)
        d = he_batch_desc()
        d.n_items, d.level, d.in_scale, d.pt_scale = B, level, in_scale, pt_scale
        d.in_ = inp.data_ptr()
        d.n_rot, d.rots, d.n_out = self._n_rot, self._rots, self._n_out
        d.pool, d.n_pool, d.pool_level = pool.data_ptr(), pool.shape[0], pool.shape[1]
        d.pt_index = self._pti
        d.out = out.data_ptr()
        h = ctypes.c_void_p()
        _check(lib().he_batch_create(ctx.h, ctypes.byref(d), flags, ctypes.byref(h)))
        self.h = h

    def run(self, stream=None):
        _check(lib().he_batch_run(self.h, _stream(stream)))

    def run_plain(self, stream=None):
        _check(lib().he_batch_run_plain(self.h, _stream(stream)))

    def info(self):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        sc = ctypes.c_double()
        _check(lib().he_batch_info(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(sc)))
        return {"rotations": a.value, "outputs": b.value, "keys": c.value, "out_scale": sc.value}

    def tuning(self):
        """MAC variant in use and the autotuner's milliseconds per variant
        (outputs per register group x polynomials per workgroup)."""
        og, ps = ctypes.c_int32(), ctypes.c_int32()
        ms = (ctypes.c_float * BATCH_MAC_VARIANTS)()
        _check(lib().he_batch_tuning(self.h, ctypes.byref(og), ctypes.byref(ps), ms, BATCH_MAC_VARIANTS))
        names = ["%dx%d" % v for v in ((4, 2), (8, 2), (16, 2), (16, 1), (32, 1))]
        return {"mac_outputs_per_group": og.value, "mac_polys_per_group": ps.value,
                "ms": {n: round(m, 3) for n, m in zip(names, ms)}}

    def close(self):
        if self.h:
            torch.cuda.synchronize()
            lib().he_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
